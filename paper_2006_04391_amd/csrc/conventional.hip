// conventional.hip -- the paper's "conventional" evaluation strategy on the
// GPU: the implicit-Euler step of the Michel-Suquet material reduced by hand
// to a scalar equation for the equivalent stress (radial return), with no
// automatic differentiation. It serves as the comparison point for the
// automatic kernel (the paper's Table "implicit_euler_timings" compares the
// strategies; the paper states that both give the same results to machine
// precision).
//
// With A_tr = C (eps - a_n) - 2/3 H D a_n, its deviator s_tr and
// q_tr = sqrt(3 J2(A_tr)): if (q_tr - sigma_y)^+ = 0 nothing flows.
// Otherwise the flow keeps the direction of s_tr and q solves
//   g(q) = q + (3 mu + H) h eps0 ((q - sigma_y) / sigma0)^n - q_tr = 0
// on (sigma_y, q_tr]; g is increasing and convex there, so Newton from q_tr
// decreases monotonically to the root. Then
//   Delta = dp 3/2 (s1, s2, s3, 2 A4, 2 A5, 2 A6)_tr / q_tr,
//   dp = h eps0 ((q - sigma_y) / sigma0)^n,
// a_{n+1} = a_n + Delta and sigma = C (eps - a_{n+1}).
//
// Consistent tangent (hand-derived from the same reduction, Section "Single
// Implicit Euler Step", the tangent of the converged step at fixed a_n).
// With the unit deviator N = s_tr / |s_tr| (tensor norm |s_tr|^2 = 2 J2),
// dp = h eps0 x^n and c = h eps0 n x^(n-1) / sigma0 (x at the converged q):
//   d Delta = 3 mu c / (1 + c (3 mu + H)) N (N : d eps)
//             + 3 mu dp / q_tr (I_dev - N (x) N) : d eps,
// so that C_tan = C - 2 mu d Delta / d eps is
//   C_tan = kappa I (x) I + 2 mu theta I_dev + 2 mu (beta - theta) N (x) N,
//   theta = 1 - 3 mu dp / q_tr,  beta = 1 - 3 mu c / (1 + c (3 mu + H)),
// kappa the bulk modulus. In engineering-shear Voigt form every entry equals
// the tensor entry (I_dev has 1/2 on the shear diagonal). For n = 1 and
// sigma_y = 0 the flow is linear in s_tr and theta = beta =
// 1 / (1 + (3 mu + H) h eps0 / sigma0) at any q_tr, q_tr = 0 included.
// Without flow C_tan = C.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "automat.h"
#include "fastmath.hpp"
#include "host_common.hpp"

namespace automat {
namespace {

constexpr int kConvBlock = 256;

struct ConvPhase {
    int32_t kind;
    double lam, mu, H, sy, s0, e0, n;
};

struct ConvArgs {
    int64_t n;
    const double *eps;
    const double *a_old;
    const uint8_t *phase;
    double *sigma;
    double *a_out;
    double *tangent;  // [36][n] row-major 6x6 per point, or null
    int32_t *iters;
    unsigned long long *nonconv;
    double h, tol;
    int32_t max_iter;
    int32_t n_phases;
    ConvPhase phases[AUTOMAT_MAX_PHASES];
};

// x^p for x > 0
__device__ __forceinline__ double powp(double x, double p) { return fm::pow_pos(x, p); }

// C_tan = kappa I (x) I + 2 mu theta I_dev + 2 mu (beta - theta) N (x) N in
// engineering-shear Voigt form, stored row-major (36 components)
__device__ __forceinline__ void store_conv_tangent(const ConvArgs &args, int64_t i, double lam,
                                                   double mu, double theta, double beta,
                                                   const double *N) {
    const int64_t n = args.n;
    const double kap = lam + 2.0 * mu / 3.0;
    const double a = 2.0 * mu * theta, b = 2.0 * mu * (beta - theta);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double v = b * N[r] * N[c];
            if (r < 3 && c < 3) v += kap + a * ((r == c ? 1.0 : 0.0) - 1.0 / 3.0);
            else if (r == c) v += 0.5 * a;
            __builtin_nontemporal_store(v, args.tangent + (6 * r + c) * n + i);
        }
}

template <bool TANGENT>
__global__ __launch_bounds__(kConvBlock) void conventional_kernel(const ConvArgs args) {
    const int64_t n = args.n;
    for (int64_t i = (int64_t)blockIdx.x * kConvBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kConvBlock) {
        double e[6], a[6];
        bool finite_in = true;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            e[c] = __builtin_nontemporal_load(args.eps + c * n + i);
            a[c] = __builtin_nontemporal_load(args.a_old + c * n + i);
            finite_in = finite_in && isfinite(e[c]) && isfinite(a[c]);
        }
        const int pid = args.phase[i];
        int status = 0;
        double sig[6];
        // tangent factors (elastic: theta = beta = 1) and the unit deviator
        double lam_t = NAN, mu_t = NAN, theta = 1.0, beta = 1.0;
        double N[6] = {0, 0, 0, 0, 0, 0};
        if (!(pid < args.n_phases) || !finite_in) {
#pragma unroll
            for (int c = 0; c < 6; ++c) sig[c] = a[c] = NAN;
            status = -1;
        } else {
            const ConvPhase p = args.phases[pid];
            const double lam = p.lam, mu = p.mu;
            // elastic stress of the strain minus a_n (engineering shears)
            double d[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) d[c] = e[c] - a[c];
            const double tr = lam * (d[0] + d[1] + d[2]);
            lam_t = lam;
            mu_t = mu;
            if (p.kind != 0) {
                // trial generalized stress A = C (eps - a_n) - 2/3 H D a_n
                double A[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) A[c] = tr + 2.0 * mu * d[c] - (2.0 / 3.0) * p.H * a[c];
#pragma unroll
                for (int c = 3; c < 6; ++c) A[c] = mu * d[c] - (1.0 / 3.0) * p.H * a[c];
                const double s0 = (2.0 * A[0] - A[1] - A[2]) * (1.0 / 3.0);
                const double s1 = (2.0 * A[1] - A[0] - A[2]) * (1.0 / 3.0);
                const double s2 = (2.0 * A[2] - A[0] - A[1]) * (1.0 / 3.0);
                const double J2 = 0.5 * (s0 * s0 + s1 * s1 + s2 * s2) + A[3] * A[3] + A[4] * A[4] +
                                  A[5] * A[5];
                const double qtr = sqrt(3.0 * J2);
                if (qtr - p.sy > 0.0 && p.e0 > 0.0) {
                    const double kap = (3.0 * mu + p.H) * args.h * p.e0;
                    const double is0 = 1.0 / p.s0;
                    double q = qtr;
                    int k = 0;
                    bool conv = false;
                    for (; k < args.max_iter; ++k) {
                        const double x = (q - p.sy) * is0;
                        const double rn1 = p.n == 1.0 ? 1.0 : powp(x, p.n - 1.0);
                        const double g = q + kap * rn1 * x - qtr;
                        const double dg = 1.0 + kap * p.n * rn1 * is0;
                        double qn = q - g / dg;
                        if (!(qn > p.sy)) qn = 0.5 * (q + p.sy);  // stay in the flow range
                        const double step = fabs(qn - q);
                        q = qn;
                        if (step <= args.tol * q) {
                            conv = true;
                            ++k;
                            break;
                        }
                    }
                    status = conv ? k : -1;
                    const double x = (q - p.sy) * is0;
                    const double rn1 = p.n == 1.0 ? 1.0 : powp(x, p.n - 1.0);
                    const double dp = args.h * p.e0 * rn1 * x;
                    const double f = 1.5 * dp / qtr;
                    if (TANGENT) {
                        const double cc = args.h * p.e0 * p.n * rn1 * is0;
                        theta = 1.0 - 3.0 * mu * dp / qtr;
                        beta = 1.0 - 3.0 * mu * cc / (1.0 + cc * (3.0 * mu + p.H));
                        const double in = 1.0 / sqrt(2.0 * J2);
                        N[0] = s0 * in;
                        N[1] = s1 * in;
                        N[2] = s2 * in;
                        N[3] = A[3] * in;
                        N[4] = A[4] * in;
                        N[5] = A[5] * in;
                    }
                    const double dlt[6] = {f * s0, f * s1, f * s2, 2.0 * f * A[3], 2.0 * f * A[4],
                                           2.0 * f * A[5]};
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        a[c] += dlt[c];
                        d[c] = e[c] - a[c];
                    }
                } else if (TANGENT && p.n == 1.0 && p.sy == 0.0 && p.e0 > 0.0) {
                    // linear flow: the tangent does not depend on q_tr
                    theta = beta = 1.0 / (1.0 + (3.0 * mu + p.H) * args.h * p.e0 / p.s0);
                }
            }
            const double t2 = lam * (d[0] + d[1] + d[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) sig[c] = t2 + 2.0 * mu * d[c];
#pragma unroll
            for (int c = 3; c < 6; ++c) sig[c] = mu * d[c];
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            __builtin_nontemporal_store(sig[c], args.sigma + c * n + i);
            if (args.a_out) __builtin_nontemporal_store(a[c], args.a_out + c * n + i);
        }
        if (TANGENT) store_conv_tangent(args, i, lam_t, mu_t, theta, beta, N);
        if (args.iters) args.iters[i] = status;
        const unsigned long long mask = __ballot(status < 0);
        if (args.nonconv && mask && (int)(threadIdx.x & 63) == __ffsll((long long)mask) - 1)
            atomicAdd(args.nonconv, (unsigned long long)__popcll(mask));
    }
}

}  // namespace
}  // namespace automat

using namespace automat;

extern "C" int32_t automat_evaluate_conventional_ex(int64_t n, const double *eps_new,
                                                    const double *a_old, const uint8_t *phase,
                                                    const automat_params *params, double h,
                                                    double tol, int32_t max_iter,
                                                    double *sigma_out, double *a_out,
                                                    double *tangent_out, int32_t *iters_out,
                                                    uint64_t *nonconverged, void *stream) {
    if (n < 0) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || !std::isfinite(tol) || !(tol > 0.0) || max_iter < 1)
        return AUTOMAT_EINVAL;
    MSGSM::Phase raw[AUTOMAT_MAX_PHASES];
    int32_t nph = 0;
    int32_t rc = copy_params(params, raw, &nph);
    if (rc) return rc;
    if (n == 0) return AUTOMAT_OK;
    if (!eps_new || !a_old || !phase || !sigma_out) return AUTOMAT_EINVAL;
    if (tangent_out && ((const void *)tangent_out == (const void *)eps_new ||
                        (const void *)tangent_out == (const void *)a_old ||
                        tangent_out == sigma_out || tangent_out == a_out))
        return AUTOMAT_EINVAL;
    ConvArgs args;
    std::memset(&args, 0, sizeof args);
    for (int k = 0; k < nph; ++k) {
        const MSGSM::Phase &q = raw[k];
        ConvPhase &c = args.phases[k];
        c.kind = q.kind;
        c.lam = q.E * q.nu / ((1.0 + q.nu) * (1.0 - 2.0 * q.nu));
        c.mu = q.E / (2.0 * (1.0 + q.nu));
        c.H = q.H;
        c.sy = q.sy;
        c.s0 = q.s0;
        c.e0 = q.e0;
        c.n = q.n;
    }
    args.n = n;
    args.eps = eps_new;
    args.a_old = a_old;
    args.phase = phase;
    args.sigma = sigma_out;
    args.a_out = a_out;
    args.tangent = tangent_out;
    args.iters = iters_out;
    args.nonconv = reinterpret_cast<unsigned long long *>(nonconverged);
    args.h = h;
    args.tol = tol;
    args.max_iter = max_iter;
    args.n_phases = nph;
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t tiles = (n + kConvBlock - 1) / kConvBlock;
    const int64_t cap = (int64_t)cus * 8;
    const int grid = (int)(tiles < cap ? tiles : cap);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (tangent_out)
        hipLaunchKernelGGL(conventional_kernel<true>, dim3(grid), dim3(kConvBlock), 0, st, args);
    else
        hipLaunchKernelGGL(conventional_kernel<false>, dim3(grid), dim3(kConvBlock), 0, st, args);
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_evaluate_conventional(int64_t n, const double *eps_new,
                                                 const double *a_old, const uint8_t *phase,
                                                 const automat_params *params, double h, double tol,
                                                 int32_t max_iter, double *sigma_out,
                                                 double *a_out, int32_t *iters_out,
                                                 uint64_t *nonconverged, void *stream) {
    return automat_evaluate_conventional_ex(n, eps_new, a_old, phase, params, h, tol, max_iter,
                                            sigma_out, a_out, nullptr, iters_out, nonconverged,
                                            stream);
}
