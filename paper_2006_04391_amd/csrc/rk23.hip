// rk23.hip -- adaptive explicit Runge-Kutta evaluation of the material law
// over one load step (the paper's Section "Rosenbrock and Runge-Kutta
// Schemes with Adaptive Step Size": the embedded Bogacki-Shampine 3(2) pair
// known from MATLAB's ode23, automatic step size control after Hairer,
// Norsett and Wanner; Section "Error Control": the error is measured on the
// stresses).
//
// On [t_n, t_n + h] the strain moves linearly from eps_n to eps_{n+1},
// eps(s) = eps_n + (s/h)(eps_{n+1} - eps_n), and the internal variables
// follow a' = f(A(eps(s), a)) with f = dPsi/dA and A = -d omega/d a, both
// from the AD layer (one reverse sweep each, no second order needed). One
// lane per point; a wave keeps stepping until a ballot shows all its lanes
// at s = h. Step: k1 (first same as last), k2 at s + dt/2, k3 at s + 3dt/4,
// y1 = y + dt (2/9 k1 + 1/3 k2 + 4/9 k3), k4 = f(s + dt, y1),
// yh = y + dt (7/24 k1 + 1/4 k2 + 1/3 k3 + 1/8 k4); with sigma = C(eps - a)
// at the start (z0) and from y1, yh at the end (z1, zh),
// err = rms_i (z1_i - zh_i) / (atol + rtol max(|z0_i|, |z1_i|)); accept if
// err <= 1; dt *= min(fmax, max(1/5, 0.9 err^(-1/3))) with fmax = 5, or 1
// after a rejection; the first try is the whole load step.
//
// The same kernel also runs the lower-order pair of the same section, ode12:
// explicit Euler embedded in Heun's method, k1 = f(s, y) (recomputed every
// step), k2 = f(s + dt, y + dt k1), y1 = y + dt/2 (k1 + k2), yh = y + dt k1,
// with the step factor 0.9 err^(-1/2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "automat.h"
#include "gsm_kernel.hpp"
#include "host_common.hpp"

namespace automat {
namespace {

using Model = MSGSM;

struct Rk23Args {
    int64_t n;
    const double *eps_n;
    const double *eps1;
    const double *a_old;
    const uint8_t *phase;
    double *sigma;
    double *a_out;
    int32_t *steps;
    unsigned long long *nonconv;
    double h, atol, rtol;
    int32_t max_steps;
    int32_t n_phases;
    Model::Phase phases[AUTOMAT_MAX_PHASES];
};

// a' at local time theta h
__device__ __forceinline__ void rk_rhs(const Model::Phase &p, const double *e0, const double *de,
                                       double theta, const double *a, double *k) {
    double e[6], A[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = e0[i] + theta * de[i];
    Model::gen_stress(p, e, a, A);
    (void)Model::psi_grad(p, A, k);
}

// sigma = d omega / d eps at local time theta h
__device__ __forceinline__ void rk_stress(const Model::Phase &p, const double *e0, const double *de,
                                          double theta, const double *a, double *z) {
    double e[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = e0[i] + theta * de[i];
    Model::stress(p, e, a, z);
}

template <bool BS23>
__global__ __launch_bounds__(kBlock) void rk_kernel(const Rk23Args args) {
    __shared__ Model::Phase tab[AUTOMAT_MAX_PHASES];
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x) {
        Model::Phase q = args.phases[k];
        Model::derive(q);
        tab[k] = q;
    }
    __syncthreads();
    const int64_t n = args.n;
    const double h = args.h, atol = args.atol, rtol = args.rtol;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n;
         base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + threadIdx.x;
        if (i >= n) continue;
        double e0[6], de[6], y[6];
        bool finite_in = true;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double a0 = args.eps_n[c * n + i], a1 = args.eps1[c * n + i];
            y[c] = args.a_old[c * n + i];
            e0[c] = a0;
            de[c] = a1 - a0;
            finite_in = finite_in && isfinite(a0) && isfinite(a1) && isfinite(y[c]);
        }
        const int pid = args.phase[i];
        const bool valid = pid < args.n_phases && finite_in;
        const Model::Phase &p = tab[valid ? pid : 0];
        const bool flow = valid && Model::flows(p);
        int status = valid ? 1 : -1;  // elastic points: one (trivial) step
        double k1[6], z0[6];
        if (flow) {
            if (BS23) rk_rhs(p, e0, de, 0.0, y, k1);
            rk_stress(p, e0, de, 0.0, y, z0);
        }
        double s = 0.0, dt = h, fmx = 5.0;
        int accepted = 0, attempts = 0;
        bool done = !flow;
        for (;;) {
            if (__ballot(!done) == 0) break;
            if (done) continue;
            if (++attempts > args.max_steps) {
                done = true;
                status = -1;
                continue;
            }
            const bool last = dt >= h - s;
            if (last) dt = h - s;
            const double th4 = last ? 1.0 : (s + dt) / h;
            double y1[6], yh[6], k4[6];
            if constexpr (BS23) {
                const double th2 = (s + 0.5 * dt) / h, th3 = (s + 0.75 * dt) / h;
                double yt[6], k2[6], k3[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) yt[c] = y[c] + 0.5 * dt * k1[c];
                rk_rhs(p, e0, de, th2, yt, k2);
#pragma unroll
                for (int c = 0; c < 6; ++c) yt[c] = y[c] + 0.75 * dt * k2[c];
                rk_rhs(p, e0, de, th3, yt, k3);
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    y1[c] = y[c] + dt * (2.0 / 9.0 * k1[c] + 1.0 / 3.0 * k2[c] + 4.0 / 9.0 * k3[c]);
                rk_rhs(p, e0, de, th4, y1, k4);
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    yh[c] = y[c] + dt * (7.0 / 24.0 * k1[c] + 0.25 * k2[c] + 1.0 / 3.0 * k3[c] +
                                         0.125 * k4[c]);
            } else {
                double k2[6];
                rk_rhs(p, e0, de, s / h, y, k1);
#pragma unroll
                for (int c = 0; c < 6; ++c) yh[c] = y[c] + dt * k1[c];
                rk_rhs(p, e0, de, th4, yh, k2);
#pragma unroll
                for (int c = 0; c < 6; ++c) y1[c] = y[c] + 0.5 * dt * (k1[c] + k2[c]);
            }
            double z1[6], zh[6];
            rk_stress(p, e0, de, th4, y1, z1);
            rk_stress(p, e0, de, th4, yh, zh);
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double r = (z1[c] - zh[c]) / (atol + rtol * fmax(fabs(z0[c]), fabs(z1[c])));
                sum += r * r;
            }
            const double err = sqrt(sum / 6.0);
            double fac = fmx;
            if (err > 0.0)
                fac = BS23 ? 0.9 * fm::exp(-fm::log(err) * (1.0 / 3.0)) : 0.9 / sqrt(err);
            fac = fmin(fmx, fmax(0.2, fac));
            if (err <= 1.0) {
                ++accepted;
                s = last ? h : s + dt;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    y[c] = y1[c];
                    if (BS23) k1[c] = k4[c];  // first same as last
                    z0[c] = z1[c];
                }
                dt *= fac;
                fmx = 5.0;
                if (last) {
                    done = true;
                    status = accepted;
                }
            } else {
                dt *= fmin(1.0, fac);
                fmx = 1.0;
            }
        }
        double sig[6];
        if (valid) {
            double e1[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) e1[c] = args.eps1[c * n + i];
            Model::stress(p, e1, y, sig);
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) sig[c] = y[c] = NAN;
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            __builtin_nontemporal_store(sig[c], args.sigma + c * n + i);
            __builtin_nontemporal_store(y[c], args.a_out + c * n + i);
        }
        if (args.steps) args.steps[i] = status;
        count_failures(args.nonconv, status < 0);
    }
}

}  // namespace
}  // namespace automat

using namespace automat;

static int32_t launch_rk(bool bs23, int64_t n, const double *eps_n, const double *eps_new,
                         const double *a_old, const uint8_t *phase, const automat_params *params,
                         double h, double atol, double rtol, int32_t max_steps, double *sigma_out,
                         double *a_out, int32_t *steps_out, uint64_t *nonconverged, void *stream) {
    if (n < 0) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || !std::isfinite(atol) || !(atol >= 0.0) ||
        !std::isfinite(rtol) || !(rtol > 0.0) || max_steps < 1)
        return AUTOMAT_EINVAL;
    Rk23Args args;
    std::memset(&args, 0, sizeof args);
    int32_t rc = copy_params(params, args.phases, &args.n_phases);
    if (rc) return rc;
    if (n == 0) return AUTOMAT_OK;
    if (!eps_n || !eps_new || !a_old || !phase || !sigma_out || !a_out) return AUTOMAT_EINVAL;
    if (a_out == eps_n || a_out == eps_new || sigma_out == a_old) return AUTOMAT_EINVAL;
    args.n = n;
    args.eps_n = eps_n;
    args.eps1 = eps_new;
    args.a_old = a_old;
    args.phase = phase;
    args.sigma = sigma_out;
    args.a_out = a_out;
    args.steps = steps_out;
    args.nonconv = reinterpret_cast<unsigned long long *>(nonconverged);
    args.h = h;
    args.atol = atol;
    args.rtol = rtol;
    args.max_steps = max_steps;
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * 4;
    const int grid = (int)(tiles < cap ? tiles : cap);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (bs23)
        hipLaunchKernelGGL(rk_kernel<true>, dim3(grid), dim3(kBlock), 0, st, args);
    else
        hipLaunchKernelGGL(rk_kernel<false>, dim3(grid), dim3(kBlock), 0, st, args);
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_evaluate_rk23(int64_t n, const double *eps_n, const double *eps_new,
                                         const double *a_old, const uint8_t *phase,
                                         const automat_params *params, double h, double atol,
                                         double rtol, int32_t max_steps, double *sigma_out,
                                         double *a_out, int32_t *steps_out,
                                         uint64_t *nonconverged, void *stream) {
    return launch_rk(true, n, eps_n, eps_new, a_old, phase, params, h, atol, rtol, max_steps,
                     sigma_out, a_out, steps_out, nonconverged, stream);
}

extern "C" int32_t automat_evaluate_rk12(int64_t n, const double *eps_n, const double *eps_new,
                                         const double *a_old, const uint8_t *phase,
                                         const automat_params *params, double h, double atol,
                                         double rtol, int32_t max_steps, double *sigma_out,
                                         double *a_out, int32_t *steps_out,
                                         uint64_t *nonconverged, void *stream) {
    return launch_rk(false, n, eps_n, eps_new, a_old, phase, params, h, atol, rtol, max_steps,
                     sigma_out, a_out, steps_out, nonconverged, stream);
}
