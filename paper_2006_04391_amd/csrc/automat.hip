// automat.hip -- gfx950 kernels and C ABI for the per-point implicit-Euler
// GSM evaluation (forward, forward + tangent) and its vector-Jacobian
// product. See include/automat.h for the contract.
//
// Launch shape: one lane per material point, wave64, 256 lanes per block.
// Fields are structure-of-arrays, so each of the 12 input and 12 output
// component streams of a wave is one contiguous 512-byte segment. The grid
// is sized to the resident capacity of the device and strides over 256-point
// tiles; every block first builds the per-phase constant table in LDS (from
// the AD Hessian of the free energy), then reuses it for all its tiles.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "automat.h"
#include "gsm_kernel.hpp"
#include "host_common.hpp"

namespace automat {

using Model = MSGSM;
using PC = PhaseConst<Model>;

struct EvalArgs {
    int64_t n;
    const double *eps;
    const double *a_old;
    const uint8_t *phase;
    double *sigma;
    double *a_out;
    double *tangent;
    int32_t *iters;
    unsigned long long *nonconv;
    double h, tol;
    int32_t max_iter;
    uint32_t flags;
    int32_t n_phases;
    int32_t reserved;
    Model::Phase phases[AUTOMAT_MAX_PHASES];
};

#ifndef AUTOMAT_EVAL_WAVES
#define AUTOMAT_EVAL_WAVES 2
#endif

template <bool TANGENT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(AUTOMAT_EVAL_WAVES)))
void gsm_eval_kernel(const EvalArgs args) {
    extern __shared__ double smem_raw[];
    // per-lane staging of eps and a_n, component-major [12][kBlock]
    double *stage = smem_raw;
    PC *tab = reinterpret_cast<PC *>(smem_raw + 12 * kBlock);
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x)
        build_phase_const<Model>(args.phases[k], tab[k], TANGENT);
    __syncthreads();

    double *eps = stage + threadIdx.x;            // eps[c * kBlock]
    double *an = stage + 6 * kBlock + threadIdx.x;  // an[c * kBlock]
    const int64_t n = args.n;
    const double h = args.h;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // Software pipelining over tiles: the inputs of the next tile are loaded
    // into registers while the current tile computes, so the load latency is
    // hidden behind the Newton work instead of stalling each tile's start.
    double nx_e[6], nx_a[6];
    int nx_p = 0;
    auto prefetch = [&](int64_t j) {
        if (j < n) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                nx_e[c] = __builtin_nontemporal_load(args.eps + c * n + j);
                nx_a[c] = __builtin_nontemporal_load(args.a_old + c * n + j);
            }
            nx_p = args.phase[j];
        }
    };
    prefetch((int64_t)blockIdx.x * kBlock + threadIdx.x);
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        if (i >= n) continue;

        bool finite_in = true;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            finite_in = finite_in && isfinite(nx_e[c]) && isfinite(nx_a[c]);
            eps[c * kBlock] = nx_e[c];
            an[c * kBlock] = nx_a[c];
        }
        const int pid = nx_p;
        prefetch(i + stride);
        const bool valid = pid < args.n_phases && finite_in;
        const PC &pc = tab[valid ? pid : 0];
        double sig[6], anew[6], C[21];
        const int status = solve_point<Model, TANGENT>(pc, valid, eps, an, h, args.tol, args.max_iter,
                                                       args.flags, sig, anew, C);
#pragma unroll
        for (int c = 0; c < 6; ++c) __builtin_nontemporal_store(sig[c], args.sigma + c * n + i);
        if (args.a_out) {
#pragma unroll
            for (int c = 0; c < 6; ++c) __builtin_nontemporal_store(anew[c], args.a_out + c * n + i);
        }
        if constexpr (TANGENT) {
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    __builtin_nontemporal_store(C[la::pk(r, c)], args.tangent + (6 * r + c) * n + i);
        }
        if (args.iters) args.iters[i] = status;
        count_failures(args.nonconv, status < 0);
    }
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------

struct DeviceInfo {
    int cus = 0;
    int blocks_fwd = 0, blocks_tan = 0;
};

static std::mutex g_mutex;
static DeviceInfo g_dev[64];
static bool g_dev_init[64];

static int32_t device_info(DeviceInfo &out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return AUTOMAT_EHIP;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_dev_init[dev]) {
        DeviceInfo d;
        if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return AUTOMAT_EHIP;
        const size_t smem = 12 * kBlock * sizeof(double) + AUTOMAT_MAX_PHASES * sizeof(PC);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.blocks_fwd, gsm_eval_kernel<false>,
                                                         kBlock, smem) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.blocks_tan, gsm_eval_kernel<true>,
                                                         kBlock, smem) != hipSuccess)
            return AUTOMAT_EHIP;
        if (d.blocks_fwd < 1) d.blocks_fwd = 1;
        if (d.blocks_tan < 1) d.blocks_tan = 1;
        g_dev[dev] = d;
        g_dev_init[dev] = true;
    }
    out = g_dev[dev];
    return AUTOMAT_OK;
}

int32_t device_cus(int *cus) {
    DeviceInfo d;
    const int32_t rc = device_info(d);
    if (rc == AUTOMAT_OK) *cus = d.cus;
    return rc;
}

static bool valid_phase(const automat_phase &p) {
    if (!(p.kind == 0 || p.kind == 1)) return false;
    if (!(p.E > 0.0) || !std::isfinite(p.E)) return false;
    if (!(p.nu > -1.0 && p.nu < 0.5)) return false;
    if (p.kind == 1) {
        if (!(p.H >= 0.0) || !std::isfinite(p.H)) return false;
        if (!(p.sigma_y >= 0.0) || !std::isfinite(p.sigma_y)) return false;
        if (!(p.sigma0 > 0.0) || !std::isfinite(p.sigma0)) return false;
        if (!(p.eps0 >= 0.0) || !std::isfinite(p.eps0)) return false;
        if (!(p.n >= 1.0) || !std::isfinite(p.n)) return false;
    }
    return true;
}

int32_t copy_params(const automat_params *params, Model::Phase *dst, int32_t *n_phases) {
    if (!params) return AUTOMAT_EINVAL;
    if (params->n_phases < 1 || params->n_phases > AUTOMAT_MAX_PHASES) return AUTOMAT_EINVAL;
    for (int k = 0; k < params->n_phases; ++k) {
        const automat_phase &p = params->phase[k];
        if (!valid_phase(p)) return AUTOMAT_EINVAL;
        Model::Phase q;
        std::memset(&q, 0, sizeof q);
        q.kind = p.kind;
        q.reserved = 0;
        q.E = p.E;
        q.nu = p.nu;
        q.H = p.kind == 1 ? p.H : 0.0;
        q.sy = p.kind == 1 ? p.sigma_y : 0.0;
        q.s0 = p.kind == 1 ? p.sigma0 : 1.0;
        q.e0 = p.kind == 1 ? p.eps0 : 0.0;
        q.n = p.kind == 1 ? p.n : 1.0;
        dst[k] = q;
    }
    for (int k = params->n_phases; k < AUTOMAT_MAX_PHASES; ++k) std::memset(&dst[k], 0, sizeof dst[k]);
    *n_phases = params->n_phases;
    return AUTOMAT_OK;
}

}  // namespace automat

using namespace automat;

extern "C" int32_t automat_evaluate_ex(int64_t n, const double *eps_new, const double *a_old,
                                       const uint8_t *phase, const automat_params *params,
                                       double h, double tol, int32_t max_iter, double *sigma_out,
                                       double *a_out, double *tangent_out, int32_t *iters_out,
                                       uint64_t *nonconverged, uint32_t flags, void *stream) {
    if (n < 0) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || !std::isfinite(tol) || !(tol > 0.0) || max_iter < 1)
        return AUTOMAT_EINVAL;
    if (flags & ~AUTOMAT_SIGMA_CRITERION) return AUTOMAT_EINVAL;
    EvalArgs args;
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
    args.h = h;
    args.tol = tol;
    args.max_iter = max_iter;
    args.flags = flags;

    DeviceInfo dev;
    rc = device_info(dev);
    if (rc) return rc;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)dev.cus * (tangent_out ? dev.blocks_tan : dev.blocks_fwd);
    const int grid = (int)(tiles < cap ? tiles : cap);
    const size_t smem = 12 * kBlock * sizeof(double) + (size_t)args.n_phases * sizeof(PC);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (tangent_out)
        hipLaunchKernelGGL(gsm_eval_kernel<true>, dim3(grid), dim3(kBlock), smem, s, args);
    else
        hipLaunchKernelGGL(gsm_eval_kernel<false>, dim3(grid), dim3(kBlock), smem, s, args);
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_evaluate(int64_t n, const double *eps_new, const double *a_old,
                                    const uint8_t *phase, const automat_params *params, double h,
                                    double tol, int32_t max_iter, double *sigma_out, double *a_out,
                                    double *tangent_out, void *stream) {
    return automat_evaluate_ex(n, eps_new, a_old, phase, params, h, tol, max_iter, sigma_out,
                               a_out, tangent_out, nullptr, nullptr, 0u, stream);
}

extern "C" const char *automat_strerror(int32_t code) {
    switch (code) {
    case AUTOMAT_OK: return "success";
    case AUTOMAT_EINVAL: return "invalid argument";
    case AUTOMAT_EHIP: return "HIP runtime or launch error";
    case AUTOMAT_ENOMEM: return "out of memory";
    case AUTOMAT_EBUDGET: return "request exceeds the memory budget";
    default: return "unknown error";
    }
}

extern "C" const char *automat_version(void) { return "automat-gfx950 0.1"; }
