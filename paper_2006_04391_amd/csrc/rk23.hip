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
// With the tangent (rk_tan_kernel), the sensitivity Y = d a / d eps_{n+1}
// (6x6, Y(0) = 0) follows Y' = Psi''(A) ((s/h) C - K Y) and is advanced with
// the same stages and the same accepted steps (the combined system of the
// paper's Theorem on differentiating an integration step); its stress-like
// image T = C ((s/h) I - Y) enters the error measure beside sigma (42
// components in the rms), and the result is C_{n+1} = C (I - Y(h)). One
// lane per point, one wave per block: the stage Hessians Psi'' sit in
// registers and Y in two LDS buffers; a step makes one pass over the six
// columns, writing the trial Y to the second buffer, and an accepted step
// swaps the buffers.
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
    double *tangent;  // [36][n] or null (rk_tan_kernel only)
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

// stage rate k = f and Psi'' (packed) at local time theta h
__device__ __forceinline__ void rk_rhs2(const Model::Phase &p, const double *e0, const double *de,
                                        double theta, const double *a, double *k, double *P) {
    double e[6], A[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = e0[i] + theta * de[i];
    Model::gen_stress(p, e, a, A);
    (void)Model::psi_grad_hess(p, A, k, P);
}

constexpr int kTanLanes = 64;  // one wave per block

// column j of one tangent stage: Kout = Psi''_m (theta C e_j - K v)
__device__ __forceinline__ void tan_stage(const PhaseConst<Model> &pc, const double *P2m, int j,
                                          double theta, const double *v, double *Kout) {
    double b[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double t = theta * pc.Cee[la::pk(q, j)];
#pragma unroll
        for (int r = 0; r < 6; ++r) t -= pc.K[la::pk(q, r)] * v[r];
        b[q] = t;
    }
    la::symv6(P2m, b, Kout);
}

template <bool BS23>
__device__ __forceinline__ void tan_column(const PhaseConst<Model> &pc, const double (*P)[21],
                                           int j, double dt, double th0, double th2, double th3,
                                           double th4, const double *Yj, double *Y1, double *Yh) {
    double K1[6], K2[6], Yt[6];
    tan_stage(pc, P[0], j, th0, Yj, K1);
    if constexpr (BS23) {
        double K3[6], K4[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) Yt[c] = Yj[c] + 0.5 * dt * K1[c];
        tan_stage(pc, P[1], j, th2, Yt, K2);
#pragma unroll
        for (int c = 0; c < 6; ++c) Yt[c] = Yj[c] + 0.75 * dt * K2[c];
        tan_stage(pc, P[2], j, th3, Yt, K3);
#pragma unroll
        for (int c = 0; c < 6; ++c)
            Y1[c] = Yj[c] + dt * (2.0 / 9.0 * K1[c] + 1.0 / 3.0 * K2[c] + 4.0 / 9.0 * K3[c]);
        tan_stage(pc, P[3], j, th4, Y1, K4);
#pragma unroll
        for (int c = 0; c < 6; ++c)
            Yh[c] = Yj[c] + dt * (7.0 / 24.0 * K1[c] + 0.25 * K2[c] + 1.0 / 3.0 * K3[c] +
                                  0.125 * K4[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) Yh[c] = Yj[c] + dt * K1[c];
        tan_stage(pc, P[1], j, th4, Yh, K2);
#pragma unroll
        for (int c = 0; c < 6; ++c) Y1[c] = Yj[c] + 0.5 * dt * (K1[c] + K2[c]);
    }
}

__device__ __forceinline__ double tan_image(const PhaseConst<Model> &pc, int i, int j, double theta,
                                            const double *v) {
    double t = theta * pc.Cee[la::pk(i, j)];
#pragma unroll
    for (int q = 0; q < 6; ++q) t -= pc.Cee[la::pk(i, q)] * v[q];
    return t;
}

// One lane per point, one wave per block. The stage Hessians stay in
// registers (the kernel may use its SIMD's whole register file, accumulation
// registers included) and the sensitivity Y in two LDS buffers: every step
// makes one pass over the six columns, reading Y from one buffer, writing
// the trial Y1 to the other and adding the columns' share to the error; an
// accepted step swaps the buffers. Y never goes to global memory; at the end
// C (I - Y) is written to the tangent output.
template <bool BS23>
__global__ __launch_bounds__(kTanLanes) __attribute__((amdgpu_waves_per_eu(1, 1)))
void rk_tan_kernel(const Rk23Args args) {
    using PC = PhaseConst<Model>;
    constexpr int NS = BS23 ? 4 : 2;
    extern __shared__ double smem_raw[];
    // Y buffers: buffer b, entry k = 6 q + j (Y_qj), lane l at [(36 b + k) 64 + l]
    double *Ybuf = smem_raw + threadIdx.x;
    PC *tab = reinterpret_cast<PC *>(smem_raw + 2 * 36 * kTanLanes);
    for (int k = threadIdx.x; k < args.n_phases; k += blockDim.x)
        build_phase_const<Model>(args.phases[k], tab[k], false);
#pragma unroll
    for (int k = 0; k < 36; ++k) Ybuf[k * kTanLanes] = 0.0;
    __syncthreads();
    const int64_t n = args.n;
    const double h = args.h, atol = args.atol, rtol = args.rtol;
    const int64_t i = (int64_t)blockIdx.x * kTanLanes + threadIdx.x;
    const bool in = i < n;
    int cur = 0;  // buffer holding Y
    double e0[6], de[6], y[6];
    bool finite_in = in;
    if (in) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double a0 = args.eps_n[c * n + i], a1 = args.eps1[c * n + i];
            y[c] = args.a_old[c * n + i];
            e0[c] = a0;
            de[c] = a1 - a0;
            finite_in = finite_in && isfinite(a0) && isfinite(a1) && isfinite(y[c]);
        }
    }
    const int pid = in ? args.phase[i] : 0;
    const bool valid = finite_in && pid < args.n_phases;
    const PC &pc = tab[valid ? pid : 0];
    const Model::Phase &p = pc.prm;
    const bool flow = valid && Model::flows(p);
    int status = valid ? 1 : -1;
    double k1[6], z0[6], P[NS][21];
    if (flow) {
        if constexpr (BS23) rk_rhs2(p, e0, de, 0.0, y, k1, P[0]);
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
        const double th0 = s / h, th4 = last ? 1.0 : (s + dt) / h;
        const double th2 = (s + 0.5 * dt) / h, th3 = (s + 0.75 * dt) / h;
        double y1[6], yh[6], k4[6];
        if constexpr (BS23) {
            double yt[6], k2[6], k3[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) yt[c] = y[c] + 0.5 * dt * k1[c];
            rk_rhs2(p, e0, de, th2, yt, k2, P[1]);
#pragma unroll
            for (int c = 0; c < 6; ++c) yt[c] = y[c] + 0.75 * dt * k2[c];
            rk_rhs2(p, e0, de, th3, yt, k3, P[2]);
#pragma unroll
            for (int c = 0; c < 6; ++c)
                y1[c] = y[c] + dt * (2.0 / 9.0 * k1[c] + 1.0 / 3.0 * k2[c] + 4.0 / 9.0 * k3[c]);
            rk_rhs2(p, e0, de, th4, y1, k4, P[3]);
#pragma unroll
            for (int c = 0; c < 6; ++c)
                yh[c] = y[c] + dt * (7.0 / 24.0 * k1[c] + 0.25 * k2[c] + 1.0 / 3.0 * k3[c] +
                                     0.125 * k4[c]);
        } else {
            double k2[6];
            rk_rhs2(p, e0, de, th0, y, k1, P[0]);
#pragma unroll
            for (int c = 0; c < 6; ++c) yh[c] = y[c] + dt * k1[c];
            rk_rhs2(p, e0, de, th4, yh, k2, P[1]);
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
        const double *Yc = Ybuf + 36 * kTanLanes * cur;
        double *Yn = Ybuf + 36 * kTanLanes * (1 - cur);
        // columns are independent: ode12 works on three at a time (more
        // independent operations in flight); ode23's four stage Hessians
        // leave registers for one
        constexpr int kColUnroll = BS23 ? 1 : 3;
#pragma unroll kColUnroll
        for (int j = 0; j < 6; ++j) {
            double Yj[6], Y1[6], Yh[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) Yj[q] = Yc[(q * 6 + j) * kTanLanes];
            tan_column<BS23>(pc, P, j, dt, th0, th2, th3, th4, Yj, Y1, Yh);
#pragma unroll
            for (int q = 0; q < 6; ++q) Yn[(q * 6 + j) * kTanLanes] = Y1[q];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const double t0 = tan_image(pc, r, j, th0, Yj);
                const double t1 = tan_image(pc, r, j, th4, Y1);
                const double tq = tan_image(pc, r, j, th4, Yh);
                const double e = (t1 - tq) * fm::rcp(atol + rtol * fmax(fabs(t0), fabs(t1)));
                sum += e * e;
            }
        }
        const double err = sqrt(sum / 42.0);
        double fac = fmx;
        if (err > 0.0)
            fac = BS23 ? 0.9 * fm::exp(-fm::log(err) * (1.0 / 3.0)) : 0.9 / sqrt(err);
        fac = fmin(fmx, fmax(0.2, fac));
        if (err <= 1.0) {
            cur = 1 - cur;
            ++accepted;
            s = last ? h : s + dt;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                y[c] = y1[c];
                if (BS23) k1[c] = k4[c];
                z0[c] = z1[c];
            }
            if constexpr (BS23) {
#pragma unroll
                for (int c = 0; c < 21; ++c) P[0][c] = P[3][c];
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
    if (!in) return;
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
    // C_{n+1} = C (I - Y(h))
    const double *Yc = Ybuf + 36 * kTanLanes * cur;
#pragma unroll 1
    for (int j = 0; j < 6; ++j) {
        double Yj[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) Yj[q] = Yc[(q * 6 + j) * kTanLanes];
#pragma unroll
        for (int r = 0; r < 6; ++r)
            __builtin_nontemporal_store(valid ? tan_image(pc, r, j, 1.0, Yj) : NAN,
                                        args.tangent + (r * 6 + j) * n + i);
    }
    if (args.steps) args.steps[i] = status;
    if (args.nonconv && status < 0) atomicAdd(args.nonconv, 1ull);
}

}  // namespace
}  // namespace automat

using namespace automat;

static int32_t launch_rk(bool bs23, int64_t n, const double *eps_n, const double *eps_new,
                         const double *a_old, const uint8_t *phase, const automat_params *params,
                         double h, double atol, double rtol, int32_t max_steps, double *sigma_out,
                         double *a_out, double *tangent_out, int32_t *steps_out,
                         uint64_t *nonconverged, void *stream) {
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
    if (tangent_out &&
        ((const void *)tangent_out == (const void *)eps_n || (const void *)tangent_out == eps_new ||
         (const void *)tangent_out == a_old || tangent_out == sigma_out || tangent_out == a_out))
        return AUTOMAT_EINVAL;
    args.n = n;
    args.eps_n = eps_n;
    args.eps1 = eps_new;
    args.a_old = a_old;
    args.phase = phase;
    args.sigma = sigma_out;
    args.a_out = a_out;
    args.tangent = tangent_out;
    args.steps = steps_out;
    args.nonconv = reinterpret_cast<unsigned long long *>(nonconverged);
    args.h = h;
    args.atol = atol;
    args.rtol = rtol;
    args.max_steps = max_steps;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (tangent_out) {
        // one wave per block: the stage Hessians in registers, the
        // sensitivity's two buffers and the phase table in LDS
        const int64_t blocks = (n + kTanLanes - 1) / kTanLanes;
        if (blocks > 0x7fffffffLL) return AUTOMAT_EINVAL;
        const size_t smem = (size_t)2 * 36 * kTanLanes * sizeof(double) +
                            (size_t)args.n_phases * sizeof(PhaseConst<Model>);
        if (bs23)
            hipLaunchKernelGGL(rk_tan_kernel<true>, dim3((unsigned)blocks), dim3(kTanLanes), smem,
                               st, args);
        else
            hipLaunchKernelGGL(rk_tan_kernel<false>, dim3((unsigned)blocks), dim3(kTanLanes), smem,
                               st, args);
        if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
        return AUTOMAT_OK;
    }
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * 4;
    const int grid = (int)(tiles < cap ? tiles : cap);
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
                     sigma_out, a_out, nullptr, steps_out, nonconverged, stream);
}

extern "C" int32_t automat_evaluate_rk12(int64_t n, const double *eps_n, const double *eps_new,
                                         const double *a_old, const uint8_t *phase,
                                         const automat_params *params, double h, double atol,
                                         double rtol, int32_t max_steps, double *sigma_out,
                                         double *a_out, int32_t *steps_out,
                                         uint64_t *nonconverged, void *stream) {
    return launch_rk(false, n, eps_n, eps_new, a_old, phase, params, h, atol, rtol, max_steps,
                     sigma_out, a_out, nullptr, steps_out, nonconverged, stream);
}

extern "C" int32_t automat_evaluate_rk23_ex(int64_t n, const double *eps_n, const double *eps_new,
                                            const double *a_old, const uint8_t *phase,
                                            const automat_params *params, double h, double atol,
                                            double rtol, int32_t max_steps, double *sigma_out,
                                            double *a_out, double *tangent_out,
                                            int32_t *steps_out, uint64_t *nonconverged,
                                            void *stream) {
    return launch_rk(true, n, eps_n, eps_new, a_old, phase, params, h, atol, rtol, max_steps,
                     sigma_out, a_out, tangent_out, steps_out, nonconverged, stream);
}

extern "C" int32_t automat_evaluate_rk12_ex(int64_t n, const double *eps_n, const double *eps_new,
                                            const double *a_old, const uint8_t *phase,
                                            const automat_params *params, double h, double atol,
                                            double rtol, int32_t max_steps, double *sigma_out,
                                            double *a_out, double *tangent_out,
                                            int32_t *steps_out, uint64_t *nonconverged,
                                            void *stream) {
    return launch_rk(false, n, eps_n, eps_new, a_old, phase, params, h, atol, rtol, max_steps,
                     sigma_out, a_out, tangent_out, steps_out, nonconverged, stream);
}
