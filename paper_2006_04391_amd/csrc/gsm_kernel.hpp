// gsm_kernel.hpp -- the per-point implicit-Euler solve shared by the
// kernels that evaluate material points (plain fields, serving batches).
// One lane per point; the point's eps and a_n are staged in LDS (stride
// kBlock) and the phase constants sit in an LDS table.
#pragma once

#include "gsm_point.hpp"

namespace automat {

constexpr int kBlock = 256;
// Newton updates after which a warm-started solve restarts from the elastic
// trial state (see solve_point)
constexpr int kWarmRestart = 6;

// Keeps the compiler from hoisting LDS reads (per-phase constants, the
// staged inputs) out of the Newton loop into registers: they are cheap to
// re-read, and holding them would cost ~90 VGPRs and most of the occupancy.
__device__ __forceinline__ void lds_reload_point() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ bool finite6(const double *x) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) ok = ok && isfinite(x[i]);
    return ok;
}

// Orders this lane's LDS writes before other lanes' later reads of them
// (the compiler would otherwise be free to reorder them; the hardware keeps
// a wave's LDS operations in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane position among the lanes of the wave whose bit is set in mask.
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Count lanes with a non-converged or invalid point, one atomic per wave.
__device__ __forceinline__ void count_failures(unsigned long long *counter, bool failed) {
    const unsigned long long mask = __ballot(failed);
    if (counter && mask) {
        const int leader = __ffsll((long long)mask) - 1;
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(counter, (unsigned long long)__popcll(mask));
    }
}

// Solve one point (all lanes of the wave call this; the Newton loop exits
// when a ballot shows every lane done). eps, an: this lane's LDS staging
// (component c at [c * S]). D: on entry the initial increment (zero, or a
// warm start such as the solution at a nearby strain), on return the
// increment a_{n+1} - a_n (zero without flow). Returns the number of Newton
// updates, or -1 (not converged within max_iter, or invalid input). Outputs
// sigma, a_{n+1} and, if TANGENT, the packed consistent tangent C[21].
// WARM: D may be non-zero on entry (otherwise it must be zero).
//
// Without TANGENT the solve keeps the Cholesky factor of the last Newton
// matrix and may take the next step with it (a simplified-Newton step),
// but only where that step is predicted to end the iteration: with
// rho = ||F_k|| / ||F_{k-1}|| the observed contraction of the last step, a
// step with a factor one step old leaves a residual of about
// 2 rho ||F_k||, and it is taken only if that meets the stopping test.
// Otherwise the Newton matrix is rebuilt at the current point, as in
// Newton's method. Likewise, a trial point is evaluated to first order
// (no Psi'') when the step changes the thermodynamic force A by less than
// 1e-3 relative: the step is then all but exact, and the next one, if any,
// is expected to reuse the factor. Both rules only skip work that the
// iteration would not use; the iterates are Newton's wherever the
// prediction fails.
template <class Model, bool TANGENT, int S = kBlock, bool WARM = false>
__device__ __forceinline__ int solve_point(const PhaseConst<Model> &pc, bool valid, const double *eps,
                                           const double *an, double h, double tol, int max_iter,
                                           unsigned flags, double *D, double *sig, double *anew,
                                           double *C) {
    const typename Model::Phase &prm = pc.prm;
    const bool newton = valid && Model::flows(prm);

    if (!newton) {
#pragma unroll
        for (int c = 0; c < 6; ++c) D[c] = 0.0;
    }
    constexpr bool kReuse = !TANGENT;
    Resid2 cur;
    // cur.M holds the Newton matrix of the current point only when have_M:
    // a trial predicted to end the iteration is evaluated to first order.
    // Otherwise (after a first-order trial) it holds the Cholesky factor of
    // the Newton matrix of an earlier iterate, valid when have_L; fprev is
    // ||F||_inf where the last step was computed.
    bool have_M = true, have_L = false;
    double fprev = 0.0;
    // merit value Phi(D) = D.K.D / 2 + h Psi(A(D)), the scale of the line
    // search's round-off allowance
    double phi = 0.0;
    int status = valid ? 0 : -1;
    if (newton) {
        residual2<Model>(prm, pc.Kinv, Strided<S>{eps}, Strided<S>{an}, D, h, cur);
        if constexpr (WARM) {
            // A guess without flow (F = D exactly: f = Psi'' = 0 there) is
            // replaced by D = 0, the elastic trial state. From the no-flow
            // side the Newton model sees no curvature, and the line search
            // would creep towards a solution across the yield surface one
            // halving at a time; from the trial state the iteration comes
            // from the flowing side, as without a warm start.
            bool nf = false;
#pragma unroll
            for (int c = 0; c < 6; ++c) nf = nf || (D[c] != 0.0);
#pragma unroll
            for (int c = 0; c < 6; ++c) nf = nf && (cur.F[c] == D[c]);
            if (nf) {
#pragma unroll
                for (int c = 0; c < 6; ++c) D[c] = 0.0;
                residual2<Model>(prm, pc.Kinv, Strided<S>{eps}, Strided<S>{an}, D, h, cur);
            }
        }
        phi = h * cur.psi;
        if constexpr (WARM) {
            double kd[6];
            la::symv6(pc.K, D, kd);
            phi += 0.5 * la::dot6(D, kd);
        }
    }
    bool done = !newton;
    int k = 0;
    // rounding level of the trial elastic strain (convergence floor below)
    double floor_F = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) floor_F = fmax(floor_F, fabs(eps[c * S] - an[c * S]));
    floor_F *= 0x1p-48;
    for (;;) {
        lds_reload_point();
        if (!done) {
            bool zero = true;
#pragma unroll
            for (int c = 0; c < 6; ++c) zero = zero && (cur.F[c] == 0.0);
            bool conv = zero;
            if (!conv) {
                if (flags & AUTOMAT_SIGMA_CRITERION) {
                    conv = k >= 1 && sigma_converged<Model>(prm, Strided<S>{eps}, Strided<S>{an},
                                                            D, cur.F, tol);
                } else {
                    // relative to the increment, or at the rounding level of
                    // the trial elastic strain that F is computed from (a flow
                    // just above the yield stress has an increment too small
                    // for the relative test to be met)
                    conv = la::norm_inf6(cur.F) <= fmax(tol * la::norm_inf6(D), floor_F);
                }
            }
            if (conv) {
                done = true;
                status = k;
            } else if (k >= max_iter) {
                done = true;
                status = -1;
            }
        }
        if (__ballot(!done) == 0) break;
        if (!done && !have_M) {
            // a first-order trial did not end the iteration: take the next
            // step with the factor at hand if it is predicted to be the
            // last, else build the Newton matrix of the current point
            bool reuse = false;
            if constexpr (kReuse) {
                const double fn = la::norm_inf6(cur.F);
                reuse = have_L &&
                        2.0 * fn * fn <= fprev * fmax(tol * la::norm_inf6(D), floor_F);
            }
            if (!reuse) {
                newton_matrix<Model>(prm, pc.Kinv, h, cur);
                have_M = true;
            }
            lds_reload_point();
        }
        bool first_order = false;
        double y[6], delta[6];
        if (!done) {
            // Cholesky factor of M = K^-1 + h Psi'' (from the last residual),
            // unless the previous factor is reused
            bool spd = true;
            if (have_M) spd = la::cholesky6(cur.M);
            have_L = spd;
#pragma unroll
            for (int c = 0; c < 6; ++c) y[c] = cur.F[c];
            la::chol_solve6(cur.M, y);
            lds_reload_point();
            if (!spd) {
                done = true;
                status = -1;
            } else {
                la::symv6(pc.Kinv, y, delta);
                if constexpr (WARM) {
                    // F = D exactly: no flow at D (f = Psi'' = 0 there), and
                    // the Newton step lands on D = 0 exactly; taken without
                    // its rounding, the next residual can be exactly zero.
                    // A warm start still unconverged after kWarmRestart
                    // updates also goes back to D = 0 (accepted without line
                    // search, below): from some starting points the line
                    // search creeps towards a solution across the yield
                    // surface, while from the elastic trial state the
                    // iteration converges as it does without a warm start.
                    bool no_flow = true;
#pragma unroll
                    for (int c = 0; c < 6; ++c) no_flow = no_flow && (cur.F[c] == D[c]);
                    if (no_flow || k == kWarmRestart) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) delta[c] = D[c];
                        have_L = false;
                    }
                }
                // quadratic convergence: a step this small relative to the
                // new iterate leaves a residual far below tol
                double dn = 0.0, nn = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    dn = fmax(dn, fabs(delta[c]));
                    nn = fmax(nn, fabs(D[c] - delta[c]));
                }
                first_order = dn <= 1e-3 * nn;
                if constexpr (kReuse) {
                    fprev = la::norm_inf6(cur.F);
                    // the step moves A by K delta = y
                    first_order = first_order ||
                                  (have_L && la::norm_inf6(y) <= 1e-3 * la::norm_inf6(cur.A));
                }
            }
        }
        // one kind of trial evaluation for the whole wave
        first_order = __ballot(!done && !first_order) == 0;
        if (!done) {
            double slope = la::dot6(cur.F, y);
            if constexpr (WARM)
                if (k == kWarmRestart) slope = -INFINITY;  // accept the restart
            const double s1 = la::dot6(D, y), s2 = la::dot6(delta, y);
            const double psi0 = cur.psi;
            // full step first; a rejected trial D - t delta moves to
            // D - t/2 delta = (D - t delta) + t/2 delta in place
            double t = 1.0, dphi;
#pragma unroll
            for (int c = 0; c < 6; ++c) D[c] -= delta[c];
            for (;;) {
                lds_reload_point();
                if (first_order)
                    residual<Model>(prm, Strided<S>{eps}, Strided<S>{an}, D, h, cur);
                else
                    residual2<Model>(prm, pc.Kinv, Strided<S>{eps}, Strided<S>{an}, D,
                                     h, cur);
                dphi = -t * s1 + 0.5 * t * t * s2 + h * (cur.psi - psi0);
                if (dphi <= -1e-4 * t * slope + 1e-13 * phi || t < 0x1p-30) break;
                t *= 0.5;
#pragma unroll
                for (int c = 0; c < 6; ++c) D[c] += t * delta[c];
            }
            have_M = !first_order;
            phi += dphi;
            if constexpr (WARM)
                if (k == kWarmRestart) phi = h * cur.psi;  // Phi(0)
            ++k;
        }
    }
    lds_reload_point();

    // outputs
    double epsv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        anew[c] = newton ? an[c * S] + D[c] : an[c * S];
        epsv[c] = eps[c * S];
    }
    if (valid) {
        Model::stress(prm, epsv, anew, sig);
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) sig[c] = anew[c] = NAN;
    }
    if constexpr (TANGENT) {
        if (newton) {
            // M at the converged point came with the last residual, unless
            // that was a first-order trial
            if (!have_M) newton_matrix<Model>(prm, pc.Kinv, h, cur);
            double *M = cur.M;
            la::cholesky6(M);
            // C = C0 + R^T M^-1 R one column of M^-1 R at a time (lower
            // triangle only: the packed result is symmetric exactly)
#pragma unroll
            for (int c = 0; c < 21; ++c) C[c] = pc.C0[c];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double x[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) x[r] = pc.R[r * 6 + j];
                la::chol_solve6(M, x);
#pragma unroll
                for (int r = j; r < 6; ++r) {
                    double acc = C[la::pk(r, j)];
#pragma unroll
                    for (int q = 0; q < 6; ++q) acc = fma(pc.R[q * 6 + r], x[q], acc);
                    C[la::pk(r, j)] = acc;
                }
            }
        } else if (valid) {
#pragma unroll
            for (int c = 0; c < 21; ++c) C[c] = pc.Cee[c];
        } else {
#pragma unroll
            for (int c = 0; c < 21; ++c) C[c] = NAN;
        }
    }
    return status;
}

}  // namespace automat
