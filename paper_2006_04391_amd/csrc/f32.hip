// f32.hip -- single-precision evaluation of the implicit-Euler GSM update
// (the paper's Section "Example", paragraph "Parallelization": single
// precision works for this material law and pays off most with tangent).
//
// Fields and arithmetic are FP32: eps, a_n in, sigma, a_{n+1} and the
// consistent tangent out, all float. The per-point algorithm is the one of
// the FP64 kernels -- Newton on F(D) = D - h f(A(a_n + D)) with the
// symmetric matrix M = K^-1 + h Psi''(A) factored by Cholesky, Armijo
// backtracking on the convex merit Phi(D) = D.K.D / 2 + h Psi(A(D)), the
// tangent C0 + R^T M^-1 R -- with the partials of omega and Psi in closed
// form (as in the semi-automatic strategy) and the convergence floor at the
// FP32 rounding level of the trial elastic strain, 16 u ||eps - a_n||_inf
// with u = 2^-23 (below it the residual carries no more digits); a Newton
// update below 8 units of rounding of the increment also ends the solve.
// One lane per point in point order; a wave leaves its Newton loop when a
// ballot shows every lane done. The per-phase constants are derived in FP64 once per
// block and kept in LDS as floats.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "automat.h"
#include "host_common.hpp"
#include "linalg6.hpp"
#include "msgsm.hpp"

namespace automat {
namespace {

constexpr int kF32Block = 256;

struct F32Args {
    int64_t n;
    const float *eps;
    const float *a_old;
    const uint8_t *phase;
    float *sigma;
    float *a_out;
    float *tangent;
    int32_t *iters;
    unsigned long long *nonconv;
    float h, tol;
    int32_t max_iter;
    int32_t n_phases;
    MSGSM::Phase phases[AUTOMAT_MAX_PHASES];
};

struct F32Const {
    int kind;
    int no_threshold;
    float lam, mu, h2, h1, sy, is0, coef, pq, n;
    float Kinv[21], K[21], Cee[21], C0[21], R[36];
};

__device__ __forceinline__ int pkf(int i, int j) {
    return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// per-phase constants, derived in FP64
__device__ void build_f32_const(const MSGSM::Phase &raw, F32Const &c) {
    MSGSM::Phase p = raw;
    MSGSM::derive(p);
    c.kind = p.kind;
    c.no_threshold = p.sy == 0.0;
    c.lam = (float)p.lam;
    c.mu = (float)p.mu;
    c.h2 = (float)((2.0 / 3.0) * p.H);
    c.h1 = (float)((1.0 / 3.0) * p.H);
    c.sy = (float)p.sy;
    c.is0 = (float)p.is0;
    c.coef = (float)p.coef;
    c.pq = (float)p.pq;
    c.n = (float)p.n;
    double C[6][6], Kaa[21], L[21], Kinv[21];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double v = 0.0;
            if (i < 3 && j < 3) v = p.lam + (i == j ? 2.0 * p.mu : 0.0);
            else if (i == j) v = p.mu;
            C[i][j] = v;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            const double hm = i == j ? (i < 3 ? 2.0 : 1.0) * (1.0 / 3.0) * p.H : 0.0;
            Kaa[la::pk(i, j)] = C[i][j] + hm;
            L[la::pk(i, j)] = Kaa[la::pk(i, j)];
            c.K[pkf(i, j)] = (float)Kaa[la::pk(i, j)];
            c.Cee[pkf(i, j)] = (float)C[i][j];
        }
    la::cholesky6(L);
    for (int j = 0; j < 6; ++j) {
        double col[6] = {0, 0, 0, 0, 0, 0};
        col[j] = 1.0;
        la::chol_solve6(L, col);
        for (int i = j; i < 6; ++i) Kinv[la::pk(i, j)] = col[i];
    }
    for (int i = 0; i < 21; ++i) c.Kinv[i] = (float)Kinv[i];
    // R = Kinv Kae with Kae = -C; C0 = Kee - Kae^T R = C - C Kinv C
    double R[36];
    for (int j = 0; j < 6; ++j) {
        double col[6], r[6];
        for (int i = 0; i < 6; ++i) col[i] = -C[i][j];
        la::symv6(Kinv, col, r);
        for (int i = 0; i < 6; ++i) R[i * 6 + j] = r[i];
    }
    for (int i = 0; i < 36; ++i) c.R[i] = (float)R[i];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += -C[k][i] * R[k * 6 + j];
            c.C0[pkf(i, j)] = (float)(C[i][j] - s);
        }
}

__device__ __forceinline__ float powf_pos(float x, float y) { return exp2f(y * log2f(x)); }

__device__ __forceinline__ void stress_f(const F32Const &c, const float *e, const float *a,
                                         float *s) {
    float d[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = e[i] - a[i];
    const float tr = c.lam * (d[0] + d[1] + d[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) s[i] = tr + 2.0f * c.mu * d[i];
#pragma unroll
    for (int i = 3; i < 6; ++i) s[i] = c.mu * d[i];
}

// Psi, f and M = Kinv + h Psi'' at a = an + D
struct RF {
    float A[6], F[6], M[21];
    float psi;
};

__device__ __forceinline__ void residual_f(const F32Const &c, const float *e, const float *an,
                                           const float *D, float h, RF &r) {
    float a[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) a[i] = an[i] + D[i];
    stress_f(c, e, a, r.A);
#pragma unroll
    for (int i = 0; i < 3; ++i) r.A[i] -= c.h2 * a[i];
#pragma unroll
    for (int i = 3; i < 6; ++i) r.A[i] -= c.h1 * a[i];
    const float third = 1.0f / 3.0f;
    float g[6];
    g[0] = (2.0f * r.A[0] - r.A[1] - r.A[2]) * third;
    g[1] = (2.0f * r.A[1] - r.A[0] - r.A[2]) * third;
    g[2] = (2.0f * r.A[2] - r.A[0] - r.A[1]) * third;
    g[3] = 2.0f * r.A[3];
    g[4] = 2.0f * r.A[4];
    g[5] = 2.0f * r.A[5];
    const float J2 = 0.5f * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + r.A[3] * r.A[3] +
                     r.A[4] * r.A[4] + r.A[5] * r.A[5];
    float val = 0.0f, a1 = 0.0f, a2 = 0.0f;
    bool live = true;
    if (c.no_threshold) {
        const float k = 3.0f * c.is0 * c.is0;
        const float u = k * J2;
        const float cc = 0.5f * c.pq;
        if (!(u > 0.0f)) {
            live = c.n == 1.0f;
            a1 = c.coef * k;
        } else {
            const float uc1 = powf_pos(u, cc - 1.0f);
            val = c.coef * uc1 * u;
            a1 = c.coef * cc * uc1 * k;
            a2 = c.coef * cc * (cc - 1.0f) * uc1 / u * k * k;
        }
    } else {
        const float q = sqrtf(3.0f * J2);
        const float x = (q - c.sy) * c.is0;
        if (!(x > 0.0f)) {
            live = false;
        } else {
            const float xn1 = powf_pos(x, c.n - 1.0f);
            const float xn = xn1 * x;
            val = c.coef * xn * x;
            const float dq = 1.5f / q;
            const float p1 = c.coef * c.pq * c.is0 * xn;
            const float p2 = c.coef * c.pq * c.is0 * c.is0 * c.n * xn1;
            a1 = p1 * dq;
            a2 = p2 * dq * dq - p1 * dq * dq / q;
        }
    }
    if (!live) a1 = a2 = 0.0f;
    r.psi = val;
#pragma unroll
    for (int i = 0; i < 6; ++i) r.F[i] = D[i] - h * a1 * g[i];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            float d2 = 0.0f;
            if (i < 3 && j < 3) d2 = (i == j ? 2.0f : -1.0f) * third;
            else if (i == j) d2 = 2.0f;
            r.M[pkf(i, j)] = c.Kinv[pkf(i, j)] + h * (a2 * g[i] * g[j] + a1 * d2);
        }
}

__device__ __forceinline__ bool chol6f(float *L, float *idg) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        float d = L[pkf(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[pkf(j, k)] * L[pkf(j, k)];
        ok = ok && (d > 0.0f);
        const float inv = rsqrtf(d);
        L[pkf(j, j)] = d * inv;
        idg[j] = inv;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            float s = L[pkf(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[pkf(i, k)] * L[pkf(j, k)];
            L[pkf(i, j)] = s * inv;
        }
    }
    return ok;
}

__device__ __forceinline__ void cholsolve6f(const float *L, const float *idg, float *b) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[pkf(i, k)] * b[k];
        b[i] = s * idg[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        float s = b[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[pkf(k, i)] * b[k];
        b[i] = s * idg[i];
    }
}

__device__ __forceinline__ void symv6f(const float *S, const float *x, float *y) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += S[pkf(i, j)] * x[j];
        y[i] = s;
    }
}

__device__ __forceinline__ float dot6f(const float *x, const float *y) {
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) s += x[i] * y[i];
    return s;
}

__device__ __forceinline__ float ninf6f(const float *x) {
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) m = fmaxf(m, fabsf(x[i]));
    return m;
}

template <bool TANGENT>
__global__ __launch_bounds__(kF32Block) void f32_kernel(const F32Args args) {
    __shared__ F32Const tab[AUTOMAT_MAX_PHASES];
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x)
        build_f32_const(args.phases[k], tab[k]);
    __syncthreads();
    const int64_t n = args.n;
    const float h = args.h;
    for (int64_t base = (int64_t)blockIdx.x * kF32Block; base < n;
         base += (int64_t)gridDim.x * kF32Block) {
        const int64_t i = base + threadIdx.x;
        const bool in_range = i < n;
        float e[6] = {0, 0, 0, 0, 0, 0}, an[6] = {0, 0, 0, 0, 0, 0};
        bool finite_in = true;
        int pid = 0;
        if (in_range) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e[c] = __builtin_nontemporal_load(args.eps + c * n + i);
                an[c] = __builtin_nontemporal_load(args.a_old + c * n + i);
                finite_in = finite_in && isfinite(e[c]) && isfinite(an[c]);
            }
            pid = args.phase[i];
        }
        const bool valid = in_range && finite_in && pid < args.n_phases;
        const F32Const &c = tab[valid ? pid : 0];
        const bool newton = valid && c.kind != 0;
        float D[6] = {0, 0, 0, 0, 0, 0};
        float floor_F = 0.0f;
#pragma unroll
        for (int q = 0; q < 6; ++q) floor_F = fmaxf(floor_F, fabsf(e[q] - an[q]));
        floor_F *= 0x1p-19f;
        RF cur;
        float phi = 0.0f;
        if (newton) {
            residual_f(c, e, an, D, h, cur);
            phi = h * cur.psi;
        }
        bool done = !newton;
        int status = valid ? 0 : -1;
        int k = 0;
        for (;;) {
            if (!done) {
                bool zero = true;
#pragma unroll
                for (int q = 0; q < 6; ++q) zero = zero && (cur.F[q] == 0.0f);
                if (zero || ninf6f(cur.F) <= fmaxf(args.tol * ninf6f(D), floor_F)) {
                    done = true;
                    status = k;
                } else if (k >= args.max_iter) {
                    done = true;
                    status = -1;
                }
            }
            if (__ballot(!done) == 0) break;
            if (done) continue;
            float L[21], idg[6], y[6], delta[6];
#pragma unroll
            for (int q = 0; q < 21; ++q) L[q] = cur.M[q];
            if (!chol6f(L, idg)) {
                done = true;
                status = -1;
                continue;
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) y[q] = cur.F[q];
            cholsolve6f(L, idg, y);
            symv6f(c.Kinv, y, delta);
            if (ninf6f(delta) <= 0x1p-21f * ninf6f(D)) {
                // the update is below 8 units of FP32 rounding of D: the
                // iterate cannot improve in this precision (for stiff
                // points, where J amplifies the rounding of F, the
                // tolerance may not be reachable)
                done = true;
                status = k;
                continue;
            }
            const float slope = dot6f(cur.F, y);
            const float s1 = dot6f(D, y), s2 = dot6f(delta, y);
            const float psi0 = cur.psi;
            float t = 1.0f, dphi;
#pragma unroll
            for (int q = 0; q < 6; ++q) D[q] -= delta[q];
            for (;;) {
                residual_f(c, e, an, D, h, cur);
                dphi = -t * s1 + 0.5f * t * t * s2 + h * (cur.psi - psi0);
                if (dphi <= -1e-4f * t * slope + 1e-6f * fabsf(phi) || t < 0x1p-20f) break;
                t *= 0.5f;
#pragma unroll
                for (int q = 0; q < 6; ++q) D[q] += t * delta[q];
            }
            phi += dphi;
            ++k;
        }
        if (!in_range) continue;
        float anew[6], sig[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) anew[q] = an[q] + D[q];
        if (valid) {
            stress_f(c, e, anew, sig);
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) sig[q] = anew[q] = NAN;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            __builtin_nontemporal_store(sig[q], args.sigma + q * n + i);
            if (args.a_out) __builtin_nontemporal_store(anew[q], args.a_out + q * n + i);
        }
        if constexpr (TANGENT) {
            float Ct[21];
            if (newton) {
                float L[21], idg[6];
#pragma unroll
                for (int q = 0; q < 21; ++q) {
                    L[q] = cur.M[q];
                    Ct[q] = c.C0[q];
                }
                chol6f(L, idg);
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    float x[6];
#pragma unroll
                    for (int r = 0; r < 6; ++r) x[r] = c.R[r * 6 + j];
                    cholsolve6f(L, idg, x);
#pragma unroll
                    for (int r = j; r < 6; ++r) {
                        float acc = Ct[pkf(r, j)];
#pragma unroll
                        for (int q = 0; q < 6; ++q) acc = fmaf(c.R[q * 6 + r], x[q], acc);
                        Ct[pkf(r, j)] = acc;
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < 21; ++q) Ct[q] = valid ? c.Cee[q] : NAN;
            }
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    __builtin_nontemporal_store(Ct[pkf(r, q)], args.tangent + (6 * r + q) * n + i);
        }
        if (args.iters) args.iters[i] = status;
        const unsigned long long mask = __ballot(status < 0);
        if (args.nonconv && mask && (int)(threadIdx.x & 63) == __ffsll((long long)mask) - 1)
            atomicAdd(args.nonconv, (unsigned long long)__popcll(mask));
    }
}

}  // namespace
}  // namespace automat

using namespace automat;

extern "C" int32_t automat_evaluate_f32(int64_t n, const float *eps_new, const float *a_old,
                                        const uint8_t *phase, const automat_params *params,
                                        double h, double tol, int32_t max_iter, float *sigma_out,
                                        float *a_out, float *tangent_out, int32_t *iters_out,
                                        uint64_t *nonconverged, void *stream) {
    if (n < 0) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || !std::isfinite(tol) || !(tol > 0.0) || max_iter < 1)
        return AUTOMAT_EINVAL;
    F32Args args;
    std::memset(&args, 0, sizeof args);
    int32_t rc = copy_params(params, args.phases, &args.n_phases);
    if (rc) return rc;
    if (n == 0) return AUTOMAT_OK;
    if (!eps_new || !a_old || !phase || !sigma_out) return AUTOMAT_EINVAL;
    args.n = n;
    args.eps = eps_new;
    args.a_old = a_old;
    args.phase = phase;
    args.sigma = sigma_out;
    args.a_out = a_out;
    args.tangent = tangent_out;
    args.iters = iters_out;
    args.nonconv = reinterpret_cast<unsigned long long *>(nonconverged);
    args.h = (float)h;
    args.tol = (float)tol;
    args.max_iter = max_iter;
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t tiles = (n + kF32Block - 1) / kF32Block;
    const int64_t cap = (int64_t)cus * 16;
    const int grid = (int)(tiles < cap ? tiles : cap);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (tangent_out)
        hipLaunchKernelGGL(f32_kernel<true>, dim3(grid), dim3(kF32Block), 0, s, args);
    else
        hipLaunchKernelGGL(f32_kernel<false>, dim3(grid), dim3(kF32Block), 0, s, args);
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}
