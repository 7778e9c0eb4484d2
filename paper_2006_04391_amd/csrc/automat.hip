// automat.hip -- gfx950 kernels and C ABI for the per-point implicit-Euler
// GSM evaluation (forward, forward + tangent) and its vector-Jacobian
// product. See include/automat.h for the contract.
//
// Launch shape: wave64, 256 lanes per block. Fields are structure-of-arrays,
// so each of the 12 input component streams of a 64-point chunk is one
// contiguous 512-byte segment. The grid is sized to the resident capacity of
// the device; every wave strides over 64-point chunks. Every block first
// builds the per-phase constant table in LDS (from the AD Hessian of the
// free energy), then reuses it for all its chunks. Points that flow are
// compacted into full waves for the Newton solve (below).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "automat.h"
#include "gsm_kernel.hpp"
#include "host_common.hpp"
#include "msgsm_hand.hpp"

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
    int32_t polarize;  // nonzero: sigma_out receives sigma - C0 eps (basic scheme)
    double lam0, mu0;  // isotropic reference medium C0 for polarize
    const double *guess;  // [6][n] initial increments of the Newton solves, or null (zero)
    double *delta_out;    // [6][n] receives a_{n+1} - a_n, or null; may equal guess
    Model::Phase phases[AUTOMAT_MAX_PHASES];
};

// sig <- sig - C0 eps for an isotropic C0 (engineering shears)
__device__ __forceinline__ void polarize6(double *sig, const double *e, double lam0, double mu0) {
    const double tr = lam0 * (e[0] + e[1] + e[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) sig[c] -= tr + 2.0 * mu0 * e[c];
#pragma unroll
    for (int c = 3; c < 6; ++c) sig[c] -= mu0 * e[c];
}

#ifndef AUTOMAT_EVAL_WAVES
#define AUTOMAT_EVAL_WAVES 2
#endif

// Wave-level compaction. Every wave walks its own sequence of 64-point
// chunks. Points without flow (elastic phase, invalid input, out of range)
// are finished at once; flowing points are queued in the wave's LDS ring
// and the Newton solve runs on 64 queued points at a time, so its lanes are
// full even where matrix and inclusion voxels alternate along a row. At the
// end the remaining queue is solved as one partial batch.
constexpr int kWaves = kBlock / 64;
constexpr int kRing = 128;  // >= 63 left over + 64 new
// ring of one wave: eps and a_n component-major [12][kRing] doubles, then
// the point index [kRing] (int64) and the phase id [kRing] (int32)
constexpr size_t kRingBytes = 12 * kRing * sizeof(double) + kRing * (sizeof(int64_t) + sizeof(int32_t));
static_assert(kRingBytes % sizeof(double) == 0, "ring keeps 8-byte alignment");

__host__ __device__ constexpr size_t eval_smem_bytes(int n_phases) {
    return kWaves * kRingBytes + (size_t)n_phases * sizeof(PC);
}

template <bool TANGENT>
__device__ __forceinline__ void store_tangent(const EvalArgs &args, int64_t i, const double *C) {
    const int64_t n = args.n;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c)
            __builtin_nontemporal_store(C[la::pk(r, c)], args.tangent + (6 * r + c) * n + i);
}

// Solve the queued points head .. head + cnt - 1 (cnt <= 64), lane l taking
// ring slot head + l, and store their results. WARM: the Newton solves start
// from args.guess and the increments go to args.delta_out (a separate
// instantiation, so the plain kernels keep their register budget).
template <class M, bool TANGENT, bool WARM>
__device__ __forceinline__ void run_batch(const EvalArgs &args, const PhaseConst<M> *tab, double *ring,
                                          const int64_t *ridx, const int32_t *rpid, uint32_t head,
                                          uint32_t cnt, int lane) {
    const uint32_t slot = (head + (uint32_t)lane) & (kRing - 1);
    const bool active = (uint32_t)lane < cnt;
    const int raw = active ? rpid[slot] : 0;
    const bool valid = active && raw < args.n_phases;  // invalid inputs carry an id past the table
    const int pid = valid ? raw : 0;
    const int64_t i = active ? ridx[slot] : 0;
    const int64_t n = args.n;
    double sig[6], anew[6], C[TANGENT ? 21 : 1], D[6] = {0, 0, 0, 0, 0, 0};
    if (WARM && args.guess && valid) {
        bool ok = true;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            D[c] = args.guess[c * n + i];
            ok = ok && isfinite(D[c]);
        }
        if (!ok) {
#pragma unroll
            for (int c = 0; c < 6; ++c) D[c] = 0.0;
        }
    }
    const int status = solve_point<M, TANGENT, kRing, WARM>(
        tab[pid], valid, ring + slot, ring + 6 * kRing + slot, args.h, args.tol, args.max_iter,
        args.flags, D, sig, anew, C);
    if (active) {
        if (args.polarize) {
            double e[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) e[c] = ring[c * kRing + slot];
            polarize6(sig, e, args.lam0, args.mu0);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) __builtin_nontemporal_store(sig[c], args.sigma + c * n + i);
        if (args.a_out) {
#pragma unroll
            for (int c = 0; c < 6; ++c) __builtin_nontemporal_store(anew[c], args.a_out + c * n + i);
        }
        if (WARM && args.delta_out) {
#pragma unroll
            for (int c = 0; c < 6; ++c) args.delta_out[c * n + i] = D[c];
        }
        if constexpr (TANGENT) store_tangent<TANGENT>(args, i, C);
        if (args.iters) args.iters[i] = status;
    }
    count_failures(args.nonconv, active && status < 0);
    wave_lds_sync();  // the slots may be refilled next
}

// M: MSGSM (partials of omega and Psi by automatic differentiation) or
// MSGSMHand (hand-derived partials, the semi-automatic strategy).
template <class M, bool TANGENT, bool WARM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(AUTOMAT_EVAL_WAVES)))
void gsm_eval_kernel(const EvalArgs args) {
    using PC = PhaseConst<M>;
    extern __shared__ double smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *ring = smem_raw + wave * (kRingBytes / sizeof(double));
    int64_t *ridx = reinterpret_cast<int64_t *>(ring + 12 * kRing);
    int32_t *rpid = reinterpret_cast<int32_t *>(ridx + kRing);
    PC *tab = reinterpret_cast<PC *>(smem_raw + kWaves * (kRingBytes / sizeof(double)));
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x)
        build_phase_const<M>(args.phases[k], tab[k], TANGENT);
    __syncthreads();

    const int64_t n = args.n;
    const int64_t chunks = (n + 63) / 64;
    const int64_t stride = (int64_t)gridDim.x * kWaves;
    // inputs of the next chunk are loaded into registers while the current
    // one is handled, so their latency hides behind the Newton work
    double nx_e[6], nx_a[6];
    int nx_p = 0;
    auto prefetch = [&](int64_t ch) {
        const int64_t j = ch * 64 + lane;
        if (ch < chunks && j < n) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                nx_e[c] = __builtin_nontemporal_load(args.eps + c * n + j);
                nx_a[c] = __builtin_nontemporal_load(args.a_old + c * n + j);
            }
            nx_p = args.phase[j];
        }
    };
    // (the tangent kernel keeps those registers for the tangent instead)
    constexpr bool kPrefetch = !TANGENT;
    // The tangent kernel writes 36 more components per point; scattered, its
    // stores cost more than the idle lanes that compaction would save.
    constexpr bool kCompact = !TANGENT;
    uint32_t head = 0, tail = 0;  // queue positions (wave-uniform), slot = pos % kRing
    int64_t ch = (int64_t)blockIdx.x * kWaves + wave;
    if (kPrefetch) prefetch(ch);
    for (;;) {
        const bool more = ch < chunks;
        if (more && !kCompact) {
            // lane order: the chunk's points go straight into ring slots
            // tail + lane (the in-range lanes are a prefix of the wave), one
            // component at a time, so nothing is held in registers
            const int64_t i = ch * 64 + lane;
            const bool in_range = i < n;
            const uint32_t slot = (tail + (uint32_t)lane) & (kRing - 1);
            if (in_range) {
                bool finite_in = true;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double v = __builtin_nontemporal_load(args.eps + c * n + i);
                    finite_in = finite_in && isfinite(v);
                    ring[c * kRing + slot] = v;
                }
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double v = __builtin_nontemporal_load(args.a_old + c * n + i);
                    finite_in = finite_in && isfinite(v);
                    ring[(6 + c) * kRing + slot] = v;
                }
                const int pid = args.phase[i];
                ridx[slot] = i;
                rpid[slot] = (pid < args.n_phases && finite_in) ? pid : AUTOMAT_MAX_PHASES;
            }
            tail += (uint32_t)__popcll(__ballot(in_range));
            ch += stride;
            wave_lds_sync();
        } else if (more) {
            const int64_t i = ch * 64 + lane;
            const bool in_range = i < n;
            double e[6], a[6];
            bool finite_in = true;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e[c] = nx_e[c];
                a[c] = nx_a[c];
                finite_in = finite_in && isfinite(e[c]) && isfinite(a[c]);
            }
            const int pid = nx_p;
            ch += stride;
            if (kPrefetch) prefetch(ch);
            const bool valid = pid < args.n_phases && finite_in;
            const PC &pc = tab[valid ? pid : 0];
            // without compaction every point of the chunk goes through the
            // batch in lane order, which keeps the output stores coalesced
            const bool queue = kCompact ? in_range && valid && M::flows(pc.prm) : in_range;
            if (kCompact && in_range && !queue) {
                // no flow: a_{n+1} = a_n, elastic stress and stiffness.
                // Ordinary (cached) stores: these points share their 64-byte
                // lines with flowing points of the same chunk, which are
                // written one Newton batch later; held in L2, the two parts
                // leave as one line. Nontemporal stores here send the
                // partial lines to memory separately, which costs write
                // traffic and time.
                double sig[6];
                if (valid) {
                    M::stress(pc.prm, e, a, sig);
                    if (args.polarize) polarize6(sig, e, args.lam0, args.mu0);
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) sig[c] = a[c] = NAN;
                }
#pragma unroll
                for (int c = 0; c < 6; ++c) args.sigma[c * n + i] = sig[c];
                if (args.a_out) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) args.a_out[c * n + i] = a[c];
                }
                if (WARM && args.delta_out) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) args.delta_out[c * n + i] = 0.0;
                }
                if constexpr (TANGENT) {
                    double C[21];
#pragma unroll
                    for (int c = 0; c < 21; ++c) C[c] = valid ? pc.Cee[c] : NAN;
                    store_tangent<TANGENT>(args, i, C);
                }
                if (args.iters) args.iters[i] = valid ? 0 : -1;
            }
            if (kCompact) count_failures(args.nonconv, in_range && !valid);
            // append the flowing points to the ring
            const uint64_t mask = __ballot(queue);
            if (queue) {
                const uint32_t pos = lane_rank(mask);
                const uint32_t slot = (tail + pos) & (kRing - 1);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    ring[c * kRing + slot] = e[c];
                    ring[(6 + c) * kRing + slot] = a[c];
                }
                ridx[slot] = i;
                rpid[slot] = valid ? pid : AUTOMAT_MAX_PHASES;
            }
            tail += (uint32_t)__popcll(mask);
            wave_lds_sync();
        }
        // a full wave of queued points, or what is left at the end
        const uint32_t cnt = tail - head;
        if (cnt >= 64 || (!more && cnt > 0)) {
            const uint32_t take = cnt < 64 ? cnt : 64;
            run_batch<M, TANGENT, WARM>(args, tab, ring, ridx, rpid, head, take, lane);
            head += take;
        }
        if (!more && tail == head) break;
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
        const size_t smem = eval_smem_bytes(AUTOMAT_MAX_PHASES);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &d.blocks_fwd, gsm_eval_kernel<Model, false, false>, kBlock, smem) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &d.blocks_tan, gsm_eval_kernel<Model, true, false>, kBlock, smem) != hipSuccess)
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

static int32_t launch_evaluate(int64_t n, const double *eps_new, const double *a_old,
                               const uint8_t *phase, const automat_params *params, double h,
                               double tol, int32_t max_iter, double *sigma_out, double *a_out,
                               double *tangent_out, int32_t *iters_out, uint64_t *nonconverged,
                               uint32_t flags, const double *pol, const double *guess,
                               double *delta_out, void *stream);

extern "C" int32_t automat_evaluate_ex(int64_t n, const double *eps_new, const double *a_old,
                                       const uint8_t *phase, const automat_params *params,
                                       double h, double tol, int32_t max_iter, double *sigma_out,
                                       double *a_out, double *tangent_out, int32_t *iters_out,
                                       uint64_t *nonconverged, uint32_t flags, void *stream) {
    return launch_evaluate(n, eps_new, a_old, phase, params, h, tol, max_iter, sigma_out, a_out,
                           tangent_out, iters_out, nonconverged, flags, nullptr, nullptr, nullptr,
                           stream);
}

namespace automat {
int32_t evaluate_polarized(int64_t n, const double *eps, const double *a_old,
                           const uint8_t *phase, const automat_params *params, double h,
                           double tol, int32_t max_iter, double lam0, double mu0, double *tau_out,
                           double *delta, uint64_t *nonconverged, void *stream) {
    const double pol[2] = {lam0, mu0};
    return launch_evaluate(n, eps, a_old, phase, params, h, tol, max_iter, tau_out, nullptr,
                           nullptr, nullptr, nonconverged, 0u, pol, delta, delta, stream);
}

int32_t evaluate_warm(int64_t n, const double *eps, const double *a_old, const uint8_t *phase,
                      const automat_params *params, double h, double tol, int32_t max_iter,
                      double *sigma_out, double *a_out, double *tangent_out, const double *guess,
                      double *delta_out, uint64_t *nonconverged, void *stream) {
    return launch_evaluate(n, eps, a_old, phase, params, h, tol, max_iter, sigma_out, a_out,
                           tangent_out, nullptr, nonconverged, 0u, nullptr, guess, delta_out,
                           stream);
}
}  // namespace automat

static int32_t launch_evaluate(int64_t n, const double *eps_new, const double *a_old,
                               const uint8_t *phase, const automat_params *params, double h,
                               double tol, int32_t max_iter, double *sigma_out, double *a_out,
                               double *tangent_out, int32_t *iters_out, uint64_t *nonconverged,
                               uint32_t flags, const double *pol, const double *guess,
                               double *delta_out, void *stream) {
    if (n < 0) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || !std::isfinite(tol) || !(tol > 0.0) || max_iter < 1)
        return AUTOMAT_EINVAL;
    if (flags & ~(AUTOMAT_SIGMA_CRITERION | AUTOMAT_HAND_PARTIALS)) return AUTOMAT_EINVAL;
    const bool hand = flags & AUTOMAT_HAND_PARTIALS;
    if (hand && (guess || delta_out || pol)) return AUTOMAT_EINVAL;
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
    if (pol) {
        args.polarize = 1;
        args.lam0 = pol[0];
        args.mu0 = pol[1];
    }
    args.guess = guess;
    args.delta_out = delta_out;

    DeviceInfo dev;
    rc = device_info(dev);
    if (rc) return rc;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    // Two (tangent: four) rounds of resident blocks: blocks that finish
    // early are replaced by the dispatcher, which evens out the end of the
    // launch (two waves share a SIMD and one of them gets issue priority).
    // Below about 24 chunks per wave in one round (some 3 million points)
    // each block's start (its phase tables) and each wave's partly filled
    // last batch cost more than the uneven end: one round.
    const int64_t chunks = (n + 63) / 64;
    const int64_t one_round = (int64_t)dev.cus * dev.blocks_fwd;
    const int rounds = chunks < 24 * one_round * kWaves ? 1 : 2;
    const int64_t cap =
        (int64_t)dev.cus * (tangent_out ? 4 * dev.blocks_tan : rounds * dev.blocks_fwd);
    const int grid = (int)(tiles < cap ? tiles : cap);
    const size_t smem = eval_smem_bytes(args.n_phases);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool warm = guess || delta_out;
    if (hand && tangent_out)
        hipLaunchKernelGGL((gsm_eval_kernel<MSGSMHand, true, false>), dim3(grid), dim3(kBlock),
                           smem, s, args);
    else if (hand)
        hipLaunchKernelGGL((gsm_eval_kernel<MSGSMHand, false, false>), dim3(grid), dim3(kBlock),
                           smem, s, args);
    else if (tangent_out && warm)
        hipLaunchKernelGGL((gsm_eval_kernel<Model, true, true>), dim3(grid), dim3(kBlock), smem, s,
                           args);
    else if (tangent_out)
        hipLaunchKernelGGL((gsm_eval_kernel<Model, true, false>), dim3(grid), dim3(kBlock), smem,
                           s, args);
    else if (warm)
        hipLaunchKernelGGL((gsm_eval_kernel<Model, false, true>), dim3(grid), dim3(kBlock), smem,
                           s, args);
    else
        hipLaunchKernelGGL((gsm_eval_kernel<Model, false, false>), dim3(grid), dim3(kBlock), smem,
                           s, args);
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
