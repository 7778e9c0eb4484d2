// backward.hip -- vector-Jacobian product of the implicit-Euler GSM step.
//
// Outputs sigma(eps, a_{n+1}) and a_{n+1}(eps, a_n), with a_{n+1} the root
// of F = a - a_n - h f(eps, a) (Section "Single Implicit Euler Step"). The
// equation solve is one elementary operation whose derivative comes from the
// implicit function theorem, and h carries no derivative (Theorem
// ad_integration_step). Given cotangents gs of sigma and ga of a_{n+1}:
//
//   abar = ga + omega_ae gs                (total cotangent of a_{n+1})
//   J^T w = abar,  J = I + h Psi'' K        (adjoint of the Newton system)
//   grad a_n   = w
//   grad eps   = omega_ee gs - omega_ea v,  v = h Psi'' w
//   grad p     = d/dp [gs . d omega/deps - v . d omega/da]   (E, nu, H)
//              + d/dp [h w . dPsi/dA]                        (sigma_y, sigma0, eps0, n)
//
// J^T = K M with the same symmetric M = K^{-1} + h Psi'' the forward solve
// factors, so w = M^{-1} K^{-1} abar (Cholesky); h Psi'' w is one more
// Hessian-vector pass (not K^{-1} abar - K^{-1} w, which cancels when the
// step is nearly elastic).
// Every second derivative is a forward-over-reverse pass of the AD layer:
// one over omega seeded with gs on eps, one over omega seeded with (gs, -v)
// and E, nu, H as leaves, one over Psi seeded with h w and its four
// parameters as leaves. Parameter cotangents are reduced per phase in LDS
// and added to the caller's array with one atomic per phase and block.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "automat.h"
#include "gsm_point.hpp"
#include "host_common.hpp"

namespace automat {

using Model = MSGSM;
using PC = PhaseConst<Model>;

namespace {

constexpr int kBlock = 256;

struct BackArgs {
    int64_t n;
    const double *eps;
    const double *a_new;
    const uint8_t *phase;
    const double *gs;
    const double *ga;
    double *geps;
    double *gan;
    double *gpar;
    double h;
    int32_t n_phases;
    int32_t reserved;
    Model::Phase phases[AUTOMAT_MAX_PHASES];
};

__global__ __launch_bounds__(kBlock) void gsm_backward_kernel(const BackArgs args) {
    __shared__ PC tab[AUTOMAT_MAX_PHASES];
    __shared__ double red[AUTOMAT_MAX_PHASES][AUTOMAT_NPAR];
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x)
        build_phase_const<Model>(args.phases[k], tab[k], false);
    for (int k = threadIdx.x; k < AUTOMAT_MAX_PHASES * AUTOMAT_NPAR; k += blockDim.x)
        red[k / AUTOMAT_NPAR][k % AUTOMAT_NPAR] = 0.0;
    __syncthreads();

    const int64_t n = args.n;
    const double h = args.h;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        if (i >= n) continue;
        double eps[6], a[6], gs[6], ga[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            eps[c] = args.eps[c * n + i];
            a[c] = args.a_new[c * n + i];
            gs[c] = args.gs ? args.gs[c * n + i] : 0.0;
            ga[c] = args.ga ? args.ga[c * n + i] : 0.0;
        }
        const int pid = args.phase[i];
        double ge[6], w[6];
        if (pid >= args.n_phases) {
#pragma unroll
            for (int c = 0; c < 6; ++c) ge[c] = w[c] = NAN;
        } else {
            const PC &pc = tab[pid];
            const Model::Phase &prm = pc.prm;
            // abar = ga + omega_ae gs
            double ee[6], ae[6];
            Model::omega_hvp_eps(prm, eps, a, gs, ee, ae);
            double abar[6], r[6], v[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) abar[c] = ga[c] + ae[c];
            double gp[AUTOMAT_NPAR] = {0, 0, 0, 0, 0, 0, 0};
            if (Model::flows(prm)) {
                double A[6], M[21];
                Model::gen_stress(prm, eps, a, A);
                Model::psi_hess(prm, A, M);
#pragma unroll
                for (int c = 0; c < 21; ++c) M[c] = pc.Kinv[c] + h * M[c];
                la::cholesky6(M);
                la::symv6(pc.Kinv, abar, r);
#pragma unroll
                for (int c = 0; c < 6; ++c) w[c] = r[c];
                la::chol_solve6(M, w);
                double hw[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) hw[c] = h * w[c];
                Model::psi_hvp(prm, A, hw, v);   // v = h Psi'' w
                Model::psi_param_partials(prm, A, hw, gp + 3);
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    w[c] = abar[c];
                    v[c] = 0.0;
                }
            }
            double mv[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) mv[c] = -v[c];
            Model::omega_hvp_params(prm, eps, a, gs, mv, ge, gp);
            for (int c = 0; c < AUTOMAT_NPAR; ++c) atomicAdd(&red[pid][c], gp[c]);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            args.geps[c * n + i] = ge[c];
            if (args.gan) args.gan[c * n + i] = w[c];
        }
    }
    __syncthreads();
    if (args.gpar) {
        for (int k = threadIdx.x; k < args.n_phases * AUTOMAT_NPAR; k += blockDim.x) {
            const double val = red[k / AUTOMAT_NPAR][k % AUTOMAT_NPAR];
            if (val != 0.0) atomicAdd(&args.gpar[k], val);
        }
    }
}

}  // namespace
}  // namespace automat

using namespace automat;

extern "C" int32_t automat_evaluate_backward(int64_t n, const double *eps_new, const double *a_old,
                                             const double *a_new, const uint8_t *phase,
                                             const automat_params *params, double h,
                                             const double *grad_sigma, const double *grad_a,
                                             double *grad_eps, double *grad_a_old,
                                             double *grad_params, void *stream) {
    if (n < 0 || !std::isfinite(h) || !(h > 0.0)) return AUTOMAT_EINVAL;
    BackArgs args;
    std::memset(&args, 0, sizeof args);
    int32_t rc = copy_params(params, args.phases, &args.n_phases);
    if (rc) return rc;
    if (n == 0) return AUTOMAT_OK;
    if (!eps_new || !a_old || !a_new || !phase || !grad_eps) return AUTOMAT_EINVAL;
    args.n = n;
    args.eps = eps_new;
    args.a_new = a_new;
    args.phase = phase;
    args.gs = grad_sigma;
    args.ga = grad_a;
    args.geps = grad_eps;
    args.gan = grad_a_old;
    args.gpar = grad_params;
    args.h = h;
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * 4;
    const int grid = (int)(tiles < cap ? tiles : cap);
    hipLaunchKernelGGL(gsm_backward_kernel, dim3(grid), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), args);
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}
