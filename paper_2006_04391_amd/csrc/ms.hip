// ms.hip -- the Moulinec-Suquet basic scheme around the material-point
// evaluation (the FFT-based homogenization of the paper's Section
// "Example", paragraph "Material Law Evaluations": one material sweep
// without tangent per fixed-point iteration).
//
// Periodic grid of nx * ny * nz voxels (x fastest), strain-controlled load
// with macroscopic strain E per step. With an isotropic reference medium
// C0 = (lambda0, mu0), one iteration is
//
//   tau     = material(eps, a_n) - C0 eps              (one evaluation sweep
//                                                       writing the polarization)
//   tau^    = FFT(tau)                                 (6 batched D2Z)
//   eps^(xi)= -Gamma0(xi) : tau^(xi), xi != 0;  eps^(0) = E
//   eps'    = IFFT(eps^) / N                           (6 batched Z2D)
//   err     = ||eps' - eps||_2 / ||E||
//
// with Gamma0_khij = [d_ki q_h q_j + d_hi q_k q_j + d_kj q_h q_i +
// d_hj q_k q_i] / (4 mu0) - (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0))
// q_i q_j q_k q_h, q = xi / |xi| (continuous operator at every xi != 0,
// including the Nyquist planes), applied as
// eps^_kh = -[(q_k v_h + q_h v_k) / (2 mu0) - c2 (q.v) q_k q_h], v = tau^ q.
// Norms are tensor norms (engineering shears count half their square), the
// L2 norm of a field is averaged over voxels. At convergence one more sweep
// at the converged strain gives the committed a_{n+1} and sigma.
// Reductions are deterministic: per-block partial sums in fixed order.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>
#include <new>

#include "automat.h"
#include "host_common.hpp"

namespace automat {
namespace {

constexpr int kRedBlock = 256;
constexpr int kRedBlocks = 1024;

struct MsField {
    int nx, ny, nz;
    int64_t n;   // real points
    int64_t nh;  // half-spectrum points nz * ny * (nx / 2 + 1)
};

__device__ __forceinline__ double freq(int k, int N) { return (double)(k <= N / 2 ? k : k - N) / N; }

// accumulate -Gamma0(q) : t for a (not necessarily unit) frequency q
__device__ __forceinline__ void gamma_add(double q1, double q2, double q3,
                                          const hipfftDoubleComplex *t, double c1, double c2,
                                          double *er, double *ei) {
    const double inv = 1.0 / sqrt(q1 * q1 + q2 * q2 + q3 * q3);
    q1 *= inv;
    q2 *= inv;
    q3 *= inv;
    // tau tensor: T11 t0, T22 t1, T33 t2, T23 t3, T13 t4, T12 t5; v = T q
    double vr[3], vi[3];
    vr[0] = t[0].x * q1 + t[5].x * q2 + t[4].x * q3;
    vi[0] = t[0].y * q1 + t[5].y * q2 + t[4].y * q3;
    vr[1] = t[5].x * q1 + t[1].x * q2 + t[3].x * q3;
    vi[1] = t[5].y * q1 + t[1].y * q2 + t[3].y * q3;
    vr[2] = t[4].x * q1 + t[3].x * q2 + t[2].x * q3;
    vi[2] = t[4].y * q1 + t[3].y * q2 + t[2].y * q3;
    const double sr = q1 * vr[0] + q2 * vr[1] + q3 * vr[2];
    const double si = q1 * vi[0] + q2 * vi[1] + q3 * vi[2];
    const double q[3] = {q1, q2, q3};
    const int K[6] = {0, 1, 2, 1, 0, 0}, Hh[6] = {0, 1, 2, 2, 2, 1};
    for (int c = 0; c < 6; ++c) {
        const int k = K[c], h = Hh[c];
        const double g = c < 3 ? 1.0 : 2.0;  // engineering shear
        er[c] -= g * (c1 * (q[k] * vr[h] + q[h] * vr[k]) - c2 * sr * q[k] * q[h]);
        ei[c] -= g * (c1 * (q[k] * vi[h] + q[h] * vi[k]) - c2 * si * q[k] * q[h]);
    }
}

// eps^ = -Gamma0 : tau^ on the half spectrum (in place); eps^(0) = E * n.
// A component k = N/2 of an even dimension stands for both +N/2 and -N/2:
// the operator is averaged over those sign choices, which keeps the
// spectrum Hermitian (and is the continuous operator on the pure Nyquist
// axes, Gamma0 being even in xi).
__global__ void gamma_kernel(hipfftDoubleComplex *spec, MsField f, double c1, double c2,
                             double E0, double E1, double E2, double E3, double E4, double E5) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= f.nh) return;
    const int nxh = f.nx / 2 + 1;
    const int kx = (int)(idx % nxh);
    const int ky = (int)((idx / nxh) % f.ny);
    const int kz = (int)(idx / ((int64_t)nxh * f.ny));
    const int64_t s = f.nh;
    if (kx == 0 && ky == 0 && kz == 0) {
        const double nn = (double)f.n;
        const double E[6] = {E0, E1, E2, E3, E4, E5};
        for (int c = 0; c < 6; ++c) {
            spec[c * s].x = E[c] * nn;
            spec[c * s].y = 0.0;
        }
        return;
    }
    const double q1 = freq(kx, f.nx), q2 = freq(ky, f.ny), q3 = freq(kz, f.nz);
    const bool n1 = (f.nx % 2 == 0) && kx == f.nx / 2;
    const bool n2 = (f.ny % 2 == 0) && ky == f.ny / 2;
    const bool n3 = (f.nz % 2 == 0) && kz == f.nz / 2;
    hipfftDoubleComplex t[6];
    for (int c = 0; c < 6; ++c) t[c] = spec[c * s + idx];
    double er[6] = {0, 0, 0, 0, 0, 0}, ei[6] = {0, 0, 0, 0, 0, 0};
    int cnt = 0;
    for (int p = 0; p < 8; ++p) {
        const double s1 = (p & 1) ? -1.0 : 1.0, s2 = (p & 2) ? -1.0 : 1.0, s3 = (p & 4) ? -1.0 : 1.0;
        if ((s1 < 0 && !n1) || (s2 < 0 && !n2) || (s3 < 0 && !n3)) continue;
        gamma_add(s1 * q1, s2 * q2, s3 * q3, t, c1, c2, er, ei);
        ++cnt;
    }
    const double w = 1.0 / cnt;
    for (int c = 0; c < 6; ++c) {
        spec[c * s + idx].x = er[c] * w;
        spec[c * s + idx].y = ei[c] * w;
    }
}

// eps' = raw / n; partial sums of the tensor norm of eps' - eps per block;
// eps <- eps'
__global__ __launch_bounds__(kRedBlock) void update_kernel(double *eps, const double *raw,
                                                           int64_t n, double *partial) {
    __shared__ double red[kRedBlock];
    const double inv = 1.0 / (double)n;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock) {
        for (int c = 0; c < 6; ++c) {
            const double nv = raw[c * n + i] * inv;
            const double d = nv - eps[c * n + i];
            acc += (c < 3 ? 1.0 : 0.5) * d * d;
            eps[c * n + i] = nv;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// per-block partial sums of 6 components of a field (for the mean)
__global__ __launch_bounds__(kRedBlock) void mean6_kernel(const double *x, int64_t n,
                                                          double *partial) {
    __shared__ double red[kRedBlock];
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kRedBlock)
            acc += x[c * n + i];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kRedBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[c * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// sum of m partials per row (rows = gridDim.x, 256 threads per row) in a
// fixed order: strided per-thread sums, then a tree over the threads, so the
// result does not depend on timing
__global__ __launch_bounds__(kRedBlock) void finish_kernel(const double *partial, int m,
                                                           double *out) {
    __shared__ double red[kRedBlock];
    double s = 0.0;
    for (int b = threadIdx.x; b < m; b += kRedBlock) s += partial[blockIdx.x * m + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// eps += dE (uniform shift of the strain field)
__global__ void shift_kernel(double *eps, int64_t n, double d0, double d1, double d2, double d3,
                             double d4, double d5) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    eps[i] += d0;
    eps[n + i] += d1;
    eps[2 * n + i] += d2;
    eps[3 * n + i] += d3;
    eps[4 * n + i] += d4;
    eps[5 * n + i] += d5;
}

// lam' = b - (C - C0) t with C the row-major 6x6 tangent field [36][n] and
// t = Gamma0 lam; the transform pipeline returns raw = -n Gamma0 lam (the
// operator kernel carries the minus sign of the forward update), so
// t = -raw / n;
// per-block partial sums of |lam' - lam|^2 and |b|^2; lam <- lam'
__global__ __launch_bounds__(kRedBlock) void adjoint_update_kernel(
    double *lam, const double *b, const double *raw, const double *C, int64_t n, double lam0,
    double mu0, double *partial) {
    __shared__ double red[2][kRedBlock];
    const double inv = 1.0 / (double)n;
    double acc = 0.0, accb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock) {
        double t[6];
        for (int c = 0; c < 6; ++c) t[c] = -raw[c * n + i] * inv;
        const double tr = lam0 * (t[0] + t[1] + t[2]);
        for (int r = 0; r < 6; ++r) {
            double ct = 0.0;
            for (int c = 0; c < 6; ++c) ct += C[(6 * r + c) * n + i] * t[c];
            const double c0t = r < 3 ? tr + 2.0 * mu0 * t[r] : mu0 * t[r];
            const double bv = b[r * n + i];
            const double nv = bv - (ct - c0t);
            const double d = nv - lam[r * n + i];
            acc += d * d;
            accb += bv * bv;
            lam[r * n + i] = nv;
        }
    }
    red[0][threadIdx.x] = acc;
    red[1][threadIdx.x] = accb;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = red[0][0];
        partial[gridDim.x + blockIdx.x] = red[1][0];
    }
}

// out = g + w / n - Gamma0 lam = g + w / n + raw / n (g may be null): the
// stress cotangent that carries the parameter and a_{k-1} sensitivities
__global__ void adjoint_sigma_kernel(double *out, const double *g, const double *raw, int64_t n,
                                     double w0, double w1, double w2, double w3, double w4,
                                     double w5) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / (double)n;
    const double w[6] = {w0, w1, w2, w3, w4, w5};
    for (int c = 0; c < 6; ++c)
        out[c * n + i] = (g ? g[c * n + i] : 0.0) + w[c] * inv + raw[c * n + i] * inv;
}

// out = g + w / n (g may be null)
__global__ void seed_kernel(double *out, const double *g, int64_t n, double w0, double w1,
                            double w2, double w3, double w4, double w5) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / (double)n;
    const double w[6] = {w0, w1, w2, w3, w4, w5};
    for (int c = 0; c < 6; ++c) out[c * n + i] = (g ? g[c * n + i] : 0.0) + w[c] * inv;
}

}  // namespace
}  // namespace automat

using namespace automat;

struct automat_ms {
    MsField f;
    automat_params params;
    automat_ms_options opts;
    double lam0, mu0;
    double E_prev[6];
    hipfftHandle fwd, inv;
    double *sig;   // [6][n] stress / polarization / raw inverse FFT output
    hipfftDoubleComplex *spec;  // [6][nh]
    double *partial;            // [6 * kRedBlocks]
    double *scal;               // [8] reduced scalars
    double *host_scal;          // pinned [8]
    // reverse step work space, allocated on first use
    double *tan;                // [36][n] consistent tangent at the converged strain
    double *lam;                // [6][n] adjoint field
    double *rhs;                // [6][n] right-hand side / scratch
    double *gs;                 // [6][n] stress cotangent
};

static int32_t ms_check_opts(const automat_ms_options *o) {
    if (!o) return AUTOMAT_EINVAL;
    if (o->max_iter < 1 || o->newton_max_iter < 1) return AUTOMAT_EINVAL;
    if (!o->fixed_iter && !(o->tol > 0.0)) return AUTOMAT_EINVAL;
    if (!(o->newton_tol > 0.0)) return AUTOMAT_EINVAL;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_create(int32_t nx, int32_t ny, int32_t nz,
                                     const automat_params *params,
                                     const automat_ms_options *opts, automat_ms **out) {
    if (!out || nx < 2 || ny < 2 || nz < 2) return AUTOMAT_EINVAL;
    *out = nullptr;
    MSGSM::Phase tmp[AUTOMAT_MAX_PHASES];
    int32_t nph = 0;
    int32_t rc = copy_params(params, tmp, &nph);
    if (rc) return rc;
    rc = ms_check_opts(opts);
    if (rc) return rc;
    automat_ms *m = new (std::nothrow) automat_ms();
    if (!m) return AUTOMAT_ENOMEM;
    m->f.nx = nx;
    m->f.ny = ny;
    m->f.nz = nz;
    m->f.n = (int64_t)nx * ny * nz;
    m->f.nh = (int64_t)(nx / 2 + 1) * ny * nz;
    m->params = *params;
    m->opts = *opts;
    std::memset(m->E_prev, 0, sizeof m->E_prev);
    // reference medium: mean of the extreme Lame constants of the phases
    double lmin = 1e300, lmax = -1e300, mmin = 1e300, mmax = -1e300;
    for (int k = 0; k < nph; ++k) {
        const double E = params->phase[k].E, nu = params->phase[k].nu;
        const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
        lmin = fmin(lmin, lam);
        lmax = fmax(lmax, lam);
        mmin = fmin(mmin, mu);
        mmax = fmax(mmax, mu);
    }
    m->lam0 = opts->lambda0 > 0.0 ? opts->lambda0 : 0.5 * (lmin + lmax);
    m->mu0 = opts->mu0 > 0.0 ? opts->mu0 : 0.5 * (mmin + mmax);
    if (!(m->mu0 > 0.0) || !(m->lam0 + 2.0 * m->mu0 / 3.0 > 0.0)) {
        delete m;
        return AUTOMAT_EINVAL;
    }
    int dims[3] = {nz, ny, nx};
    int dims_c[3] = {nz, ny, nx / 2 + 1};
    const size_t nb = (size_t)m->f.n * 6 * sizeof(double);
    const size_t nc = (size_t)m->f.nh * 6 * sizeof(hipfftDoubleComplex);
    bool ok = hipMalloc(&m->sig, nb) == hipSuccess &&
              hipMalloc(&m->spec, nc) == hipSuccess &&
              hipMalloc(&m->partial, 6 * kRedBlocks * sizeof(double)) == hipSuccess &&
              hipMalloc(&m->scal, 8 * sizeof(double)) == hipSuccess &&
              hipHostMalloc(&m->host_scal, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipfftPlanMany(&m->fwd, 3, dims, dims, 1, (int)m->f.n, dims_c, 1, (int)m->f.nh,
                              HIPFFT_D2Z, 6) == HIPFFT_SUCCESS;
    ok = ok && hipfftPlanMany(&m->inv, 3, dims, dims_c, 1, (int)m->f.nh, dims, 1, (int)m->f.n,
                              HIPFFT_Z2D, 6) == HIPFFT_SUCCESS;
    if (!ok) {
        automat_ms_destroy(m);
        return AUTOMAT_ENOMEM;
    }
    *out = m;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_destroy(automat_ms *m) {
    if (!m) return AUTOMAT_OK;
    if (m->fwd) (void)hipfftDestroy(m->fwd);
    if (m->inv) (void)hipfftDestroy(m->inv);
    if (m->sig) (void)hipFree(m->sig);
    if (m->spec) (void)hipFree(m->spec);
    if (m->partial) (void)hipFree(m->partial);
    if (m->scal) (void)hipFree(m->scal);
    if (m->host_scal) (void)hipHostFree(m->host_scal);
    if (m->tan) (void)hipFree(m->tan);
    if (m->lam) (void)hipFree(m->lam);
    if (m->rhs) (void)hipFree(m->rhs);
    if (m->gs) (void)hipFree(m->gs);
    delete m;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_reference(const automat_ms *m, double *lambda0, double *mu0) {
    if (!m || !lambda0 || !mu0) return AUTOMAT_EINVAL;
    *lambda0 = m->lam0;
    *mu0 = m->mu0;
    return AUTOMAT_OK;
}

static double tensor_norm(const double *e) {
    return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2] +
                0.5 * (e[3] * e[3] + e[4] * e[4] + e[5] * e[5]));
}

extern "C" int32_t automat_ms_step(automat_ms *m, const uint8_t *phase, const double *E_macro,
                                   double h, double *eps, double *a, double *sigma_out,
                                   double *sigma_mean, int32_t *iters, double *residual,
                                   void *stream) {
    if (!m || !phase || !E_macro || !eps || !a) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0)) return AUTOMAT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = m->f.n;
    const int tb = 256;
    const int gb = (int)((n + tb - 1) / tb);
    if (hipfftSetStream(m->fwd, s) != HIPFFT_SUCCESS || hipfftSetStream(m->inv, s) != HIPFFT_SUCCESS)
        return AUTOMAT_EHIP;
    // initial guess: previous strain field shifted by the macro increment
    double d[6];
    for (int c = 0; c < 6; ++c) d[c] = E_macro[c] - m->E_prev[c];
    hipLaunchKernelGGL(shift_kernel, dim3(gb), dim3(tb), 0, s, eps, n, d[0], d[1], d[2], d[3],
                       d[4], d[5]);
    const double En = fmax(tensor_norm(E_macro), 1e-300);
    const double c1 = 1.0 / (2.0 * m->mu0);
    const double c2 = (m->lam0 + m->mu0) / (m->mu0 * (m->lam0 + 2.0 * m->mu0));
    const int nhb = (int)((m->f.nh + tb - 1) / tb);
    const int rb = (int)((n + kRedBlock - 1) / kRedBlock) < kRedBlocks
                       ? (int)((n + kRedBlock - 1) / kRedBlock)
                       : kRedBlocks;
    int it = 0;
    double err = 0.0;
    int32_t rc = AUTOMAT_OK;
    for (it = 1; it <= m->opts.max_iter; ++it) {
        // material sweep writing the polarization tau = sigma - C0 eps
        rc = evaluate_polarized(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                                m->opts.newton_max_iter, m->lam0, m->mu0, m->sig, stream);
        if (rc) return rc;
        if (hipfftExecD2Z(m->fwd, m->sig, m->spec) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
        hipLaunchKernelGGL(gamma_kernel, dim3(nhb), dim3(tb), 0, s, m->spec, m->f, c1, c2,
                           E_macro[0], E_macro[1], E_macro[2], E_macro[3], E_macro[4], E_macro[5]);
        if (hipfftExecZ2D(m->inv, m->spec, m->sig) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
        hipLaunchKernelGGL(update_kernel, dim3(rb), dim3(kRedBlock), 0, s, eps, m->sig, n,
                           m->partial);
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kRedBlock), 0, s, m->partial, rb, m->scal);
        if (!m->opts.fixed_iter) {
            if (hipMemcpyAsync(m->host_scal, m->scal, sizeof(double), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return AUTOMAT_EHIP;
            err = sqrt(m->host_scal[0] / (double)n) / En;
            if (err <= m->opts.tol) break;
        }
    }
    if (it > m->opts.max_iter) it = m->opts.max_iter;
    if (m->opts.fixed_iter) {
        if (hipMemcpyAsync(m->host_scal, m->scal, sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return AUTOMAT_EHIP;
        err = sqrt(m->host_scal[0] / (double)n) / En;
    }
    // commit: sweep at the converged strain, a_n <- a_{n+1}
    double *sig = sigma_out ? sigma_out : m->sig;
    rc = automat_evaluate_ex(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                             m->opts.newton_max_iter, sig, a, nullptr, nullptr, nullptr, 0u,
                             stream);
    if (rc) return rc;
    if (sigma_mean) {
        hipLaunchKernelGGL(mean6_kernel, dim3(rb), dim3(kRedBlock), 0, s, sig, n, m->partial);
        hipLaunchKernelGGL(finish_kernel, dim3(6), dim3(kRedBlock), 0, s, m->partial, rb, m->scal);
        if (hipMemcpyAsync(m->host_scal, m->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return AUTOMAT_EHIP;
        for (int c = 0; c < 6; ++c) sigma_mean[c] = m->host_scal[c] / (double)n;
    }
    for (int c = 0; c < 6; ++c) m->E_prev[c] = E_macro[c];
    if (iters) *iters = it;
    if (residual) *residual = err;
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_set_macro(automat_ms *m, const double *E_prev) {
    if (!m || !E_prev) return AUTOMAT_EINVAL;
    for (int c = 0; c < 6; ++c) m->E_prev[c] = E_prev[c];
    return AUTOMAT_OK;
}

// The Green operator applied to a stress-like field x (not modified): the
// raw inverse transform, -n Gamma0 x (zero mean), lands in m->sig.
static int32_t ms_gamma(automat_ms *m, const double *x, hipStream_t s) {
    const int tb = 256;
    const int nhb = (int)((m->f.nh + tb - 1) / tb);
    const double c1 = 1.0 / (2.0 * m->mu0);
    const double c2 = (m->lam0 + m->mu0) / (m->mu0 * (m->lam0 + 2.0 * m->mu0));
    if (hipMemcpyAsync(m->sig, x, (size_t)m->f.n * 6 * sizeof(double), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        return AUTOMAT_EHIP;
    if (hipfftExecD2Z(m->fwd, m->sig, m->spec) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
    hipLaunchKernelGGL(gamma_kernel, dim3(nhb), dim3(tb), 0, s, m->spec, m->f, c1, c2, 0.0, 0.0,
                       0.0, 0.0, 0.0, 0.0);
    if (hipfftExecZ2D(m->inv, m->spec, m->sig) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_adjoint_step(automat_ms *m, const uint8_t *phase, double h,
                                           const double *eps, const double *a_prev,
                                           const double *a_next, const double *w,
                                           const double *grad_sigma, const double *grad_a,
                                           double *grad_E, double *grad_a_prev,
                                           double *grad_params, int32_t *iters, double *residual,
                                           void *stream) {
    if (!m || !phase || !eps || !a_prev || !a_next || !grad_E) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0)) return AUTOMAT_EINVAL;
    if (grad_a_prev && (grad_a_prev == grad_a || grad_a_prev == a_prev || grad_a_prev == a_next ||
                        grad_a_prev == eps))
        return AUTOMAT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = m->f.n;
    const size_t fb = (size_t)n * 6 * sizeof(double);
    if (!m->tan) {
        if (hipMalloc(&m->tan, 6 * fb) != hipSuccess || hipMalloc(&m->lam, fb) != hipSuccess ||
            hipMalloc(&m->rhs, fb) != hipSuccess || hipMalloc(&m->gs, fb) != hipSuccess) {
            (void)hipGetLastError();
            return AUTOMAT_ENOMEM;
        }
    }
    if (hipfftSetStream(m->fwd, s) != HIPFFT_SUCCESS || hipfftSetStream(m->inv, s) != HIPFFT_SUCCESS)
        return AUTOMAT_EHIP;
    const int tb = 256;
    const int gb = (int)((n + tb - 1) / tb);
    const int rb = (int)((n + kRedBlock - 1) / kRedBlock) < kRedBlocks
                       ? (int)((n + kRedBlock - 1) / kRedBlock)
                       : kRedBlocks;
    const double wz[6] = {0, 0, 0, 0, 0, 0};
    const double *wv = w ? w : wz;
    // consistent tangent field at the converged strain (a_{k-1} fixed)
    int32_t rc = automat_evaluate_ex(n, eps, a_prev, phase, &m->params, h, m->opts.newton_tol,
                                     m->opts.newton_max_iter, m->lam, nullptr, m->tan, nullptr,
                                     nullptr, 0u, stream);
    if (rc) return rc;
    // stress cotangent of the functional: g + w / n
    hipLaunchKernelGGL(seed_kernel, dim3(gb), dim3(tb), 0, s, m->gs, grad_sigma, n, wv[0], wv[1],
                       wv[2], wv[3], wv[4], wv[5]);
    // b = direct strain cotangent of the point map (backward kernel)
    rc = automat_evaluate_backward(n, eps, a_prev, a_next, phase, &m->params, h, m->gs, grad_a,
                                   m->rhs, nullptr, nullptr, stream);
    if (rc) return rc;
    // lam = b - (C - C0) Gamma0 lam, from lam = b
    if (hipMemcpyAsync(m->lam, m->rhs, fb, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return AUTOMAT_EHIP;
    int it = 0;
    double err = 0.0;
    for (it = 1; it <= m->opts.max_iter; ++it) {
        rc = ms_gamma(m, m->lam, s);
        if (rc) return rc;
        hipLaunchKernelGGL(adjoint_update_kernel, dim3(rb), dim3(kRedBlock), 0, s, m->lam, m->rhs,
                           m->sig, m->tan, n, m->lam0, m->mu0, m->partial);
        hipLaunchKernelGGL(finish_kernel, dim3(2), dim3(kRedBlock), 0, s, m->partial, rb, m->scal);
        if (!m->opts.fixed_iter || it == m->opts.max_iter) {
            if (hipMemcpyAsync(m->host_scal, m->scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return AUTOMAT_EHIP;
            err = m->host_scal[1] > 0.0 ? sqrt(m->host_scal[0] / m->host_scal[1]) : 0.0;
            if (!m->opts.fixed_iter && err <= m->opts.tol) break;
        }
    }
    if (it > m->opts.max_iter) it = m->opts.max_iter;
    // dL/dE = sum_x lam(x)
    hipLaunchKernelGGL(mean6_kernel, dim3(rb), dim3(kRedBlock), 0, s, m->lam, n, m->partial);
    hipLaunchKernelGGL(finish_kernel, dim3(6), dim3(kRedBlock), 0, s, m->partial, rb, m->scal);
    if (hipMemcpyAsync(m->host_scal, m->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AUTOMAT_EHIP;
    for (int c = 0; c < 6; ++c) grad_E[c] = m->host_scal[c];
    if (grad_a_prev || grad_params) {
        // stress cotangent g + w / n - Gamma0 lam, then the point VJP
        rc = ms_gamma(m, m->lam, s);
        if (rc) return rc;
        hipLaunchKernelGGL(adjoint_sigma_kernel, dim3(gb), dim3(tb), 0, s, m->gs, grad_sigma,
                           m->sig, n, wv[0], wv[1], wv[2], wv[3], wv[4], wv[5]);
        rc = automat_evaluate_backward(n, eps, a_prev, a_next, phase, &m->params, h, m->gs, grad_a,
                                       m->rhs, grad_a_prev, grad_params, stream);
        if (rc) return rc;
    }
    if (iters) *iters = it;
    if (residual) *residual = err;
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}
