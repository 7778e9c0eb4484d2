// ms.hip -- the Moulinec-Suquet basic scheme around the material-point
// evaluation (the FFT-based homogenization of the paper's Section
// "Example", paragraph "Material Law Evaluations": one material sweep
// without tangent per fixed-point iteration).
//
// Periodic grid of nx * ny * nz voxels (x fastest). With an isotropic
// reference medium C0 = (lambda0, mu0), one iteration is
//
//   tau     = material(eps, a_n) - C0 eps              (one evaluation sweep
//                                                       writing the polarization)
//   tau^    = FFT(tau)                                 (6 fields)
//   eps^(xi)= -Gamma0(xi) : tau^(xi), xi != 0;  eps^(0) = E
//   eps'    = IFFT(eps^) / N
//   err     = ||eps' - eps||_2 / ||E||
//
// The transforms: on grids with 128 x 128 planes, plane transforms of our
// own (slab_fft.hpp) with the strain update and its norm in the inverse
// pass, and along z either one kernel with Gamma0 between the forward and
// inverse transforms (nz = 128) or hipFFT with gamma_kernel between; on
// grids with nz = 150, 2-D hipFFT transforms in-plane and one kernel along
// z with Gamma0 (zfft150.hpp); otherwise 6-batch 3-D hipFFT plans with
// gamma_kernel and update_kernel. While the host reads an iteration's norm
// for the convergence test, the next iteration's sweep already runs.
//
// with Gamma0_khij = [d_ki q_h q_j + d_hi q_k q_j + d_kj q_h q_i +
// d_hj q_k q_i] / (4 mu0) - (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0))
// q_i q_j q_k q_h, q = xi / |xi|, applied as
// eps^_kh = -[(q_k v_h + q_h v_k) / (2 mu0) - c2 (q.v) q_k q_h], v = tau^ q.
// Where a Nyquist index N/2 of an even dimension meets another non-zero
// component, +N/2 and -N/2 are one index but different directions; there
// Gamma0 is the reference compliance C0^-1, so the converged stress has no
// content at those frequencies and the fixed point does not depend on C0.
//
// Mixed boundary conditions (the paper's uniaxial tension-compression test):
// components in the stress-controlled set take the macroscopic stress
// S_bar, the others the macroscopic strain E_bar; the zero frequency of
// every update is the E that makes the reference medium's mean stress meet
// the targets, mean(tau) + C0 E = S_bar on the stress-controlled set, solved
// in closed form on the device from tau^(0) = n mean(tau).
// Reference update (the paper's per-load-step reference stiffness): a sweep
// with tangent at the step's initial guess; C0 takes the means of the
// smallest and largest Lame constants of the isotropic parts of the tangents
// (3K = C:(I x I)/3 over the normal block, 10 mu = C_ijij - 3K).
// Norms are tensor norms (engineering shears count half their square), the
// L2 norm of a field is averaged over voxels. At convergence one more sweep
// at the converged strain gives the committed a_{n+1} and sigma.
// Reductions are deterministic: per-block partial sums in fixed order.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <mutex>

#include <cmath>
#include <cstring>
#include <new>

#include "automat.h"
#include "host_common.hpp"
#include "slab_fft.hpp"
#include "zfft150.hpp"

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

// Zero-frequency data of one update: the prescribed strain (E) and stress
// (S) and the stress-controlled set (bit c of mask); Eout receives the
// macroscopic strain of the update (device).
struct MacroBC {
    double E[6], S[6];
    uint32_t mask;
    double *Eout;
};

// E with E_c = Ebar_c off the stress-controlled set and
// (C0 E)_c = r_c on it, for the isotropic C0 = (lam, mu) in engineering
// Voigt form. Shears decouple (mu E_c = r_c); the m stress-controlled
// normal components x_i solve lam (K + X) + 2 mu x_i = r_i with K the sum of
// the prescribed normal strains and X = sum x_i, so
// X = (sum r_i - m lam K) / (m lam + 2 mu).
__host__ __device__ inline void mixed_solve(double lam, double mu, uint32_t mask,
                                            const double *Ebar, const double *r, double *E) {
    double K = 0.0, R = 0.0;
    int m = 0;
    for (int c = 0; c < 3; ++c) {
        if (mask >> c & 1u) {
            ++m;
            R += r[c];
        } else {
            K += Ebar[c];
        }
    }
    const double X = m ? (R - m * lam * K) / (m * lam + 2.0 * mu) : 0.0;
    for (int c = 0; c < 3; ++c)
        E[c] = (mask >> c & 1u) ? (r[c] - lam * (K + X)) / (2.0 * mu) : Ebar[c];
    for (int c = 3; c < 6; ++c) E[c] = (mask >> c & 1u) ? r[c] / mu : Ebar[c];
}

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

// The zero frequency: t holds tau^(0) = n mean(tau) in, E n out (the
// macroscopic strain of the update, also written to bc.Eout).
__device__ __forceinline__ void gamma_zero(hipfftDoubleComplex *t, const MsField &f, double lam0,
                                           double mu0, const MacroBC &bc) {
    const double nn = (double)f.n;
    double r[6], E[6];
    for (int c = 0; c < 6; ++c) r[c] = bc.S[c] - t[c].x / nn;
    mixed_solve(lam0, mu0, bc.mask, bc.E, r, E);
    for (int c = 0; c < 6; ++c) {
        t[c].x = E[c] * nn;
        t[c].y = 0.0;
        if (bc.Eout) bc.Eout[c] = E[c];
    }
}

// eps^ = -Gamma0 : tau^ at the non-zero frequency (kx, ky, kz), in place
__device__ __forceinline__ void gamma_point(hipfftDoubleComplex *t, const MsField &f, int kx,
                                            int ky, int kz, double lam0, double mu0) {
    const bool n1 = (f.nx % 2 == 0) && kx == f.nx / 2;
    const bool n2 = (f.ny % 2 == 0) && ky == f.ny / 2;
    const bool n3 = (f.nz % 2 == 0) && kz == f.nz / 2;
    const int nonzero = (kx != 0) + (ky != 0) + (kz != 0);
    double er[6] = {0, 0, 0, 0, 0, 0}, ei[6] = {0, 0, 0, 0, 0, 0};
    if ((n1 || n2 || n3) && nonzero >= 2) {
        // -C0^-1 : t; normal strains (t_i - lam0 / (3 lam0 + 2 mu0) tr t) / (2 mu0),
        // engineering shears t_c / mu0
        const double g = lam0 / (3.0 * lam0 + 2.0 * mu0);
        const double trr = t[0].x + t[1].x + t[2].x, tri = t[0].y + t[1].y + t[2].y;
        for (int c = 0; c < 3; ++c) {
            er[c] = -(t[c].x - g * trr) / (2.0 * mu0);
            ei[c] = -(t[c].y - g * tri) / (2.0 * mu0);
        }
        for (int c = 3; c < 6; ++c) {
            er[c] = -t[c].x / mu0;
            ei[c] = -t[c].y / mu0;
        }
    } else {
        const double c1 = 1.0 / (2.0 * mu0);
        const double c2 = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
        gamma_add(freq(kx, f.nx), freq(ky, f.ny), freq(kz, f.nz), t, c1, c2, er, ei);
    }
    for (int c = 0; c < 6; ++c) {
        t[c].x = er[c];
        t[c].y = ei[c];
    }
}

// eps^ = -Gamma0 : tau^ on the half spectrum (in place); eps^(0) = E * n
// with E from the macroscopic conditions (above).
// Value c of frequency (kx, ky, kz) sits at spec[c * cs + kz * zs + ky * nxh
// + kx]: cs = nh, zs = ny * nxh for component-major spectra (the 3-D
// transforms), cs = ny * nxh, zs = 6 cs for plane-major ones (the slab
// transforms).
__global__ void gamma_kernel(hipfftDoubleComplex *spec, MsField f, double lam0, double mu0,
                             MacroBC bc, int64_t cs, int64_t zs) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= f.nh) return;
    const int nxh = f.nx / 2 + 1;
    const int kx = (int)(idx % nxh);
    const int ky = (int)((idx / nxh) % f.ny);
    const int kz = (int)(idx / ((int64_t)nxh * f.ny));
    const int64_t at = (int64_t)kz * zs + (int64_t)ky * nxh + kx;
    hipfftDoubleComplex t[6];
    for (int c = 0; c < 6; ++c) t[c] = spec[c * cs + at];
    if (kx == 0 && ky == 0 && kz == 0)
        gamma_zero(t, f, lam0, mu0, bc);
    else
        gamma_point(t, f, kx, ky, kz, lam0, mu0);
    for (int c = 0; c < 6; ++c) spec[c * cs + at] = t[c];
}

// The transforms along z (length 128) with Gamma0 between them, for the
// plane-major spectra of 128^3 grids: a work-group takes kZR = 4
// consecutive in-plane frequencies r = ky * 65 + kx with all six
// components (24 columns of 128 values, 8 lanes each: the radix-16 and
// radix-8 passes of slab_fft.hpp), keeps them in LDS between the forward
// transform, the Green operator (the six components of one frequency
// together) and the inverse transform, and writes them back in place.
// Neighbouring work-groups share 128-byte lines, so each XCD walks a
// contiguous range of groups (xcd_group).
// Group of block b when blocks go to the eight XCDs in turn: XCD b mod 8
// walks a contiguous range of the G groups (a bijection for any G).
__device__ __forceinline__ int xcd_group(int b, int G) {
    const int q = G / 8, rem = G % 8, x = b % 8;
    return x * q + (x < rem ? x : rem) + b / 8;
}

constexpr int kZR = 4;
constexpr int kZThreads = 6 * kZR * 8;
constexpr int kZLD = slab::N + 1;
__global__ __launch_bounds__(kZThreads) void z_gamma_kernel(slab::cd *spec, MsField f,
                                                            double lam0, double mu0, MacroBC bc) {
    using slab::cd;
    __shared__ cd X[6 * kZR * kZLD];
    __shared__ cd tw[slab::N];
    slab::init_twiddles(tw);
    const int grp = xcd_group((int)blockIdx.x, (int)gridDim.x);
    const int64_t P = (int64_t)slab::N * slab::NH;
    const int r0 = grp * kZR;
    const int t = threadIdx.x;
    const int rr = t & (kZR - 1), l = (t / kZR) & 7, c = t / (kZR * 8);
    const int col = c * kZR + rr;
    cd *base = spec + (int64_t)c * P + r0 + rr;  // + z * 6 P
    __syncthreads();
    {
        cd v[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) v[n1] = base[(int64_t)(8 * n1 + l) * 6 * P];
        slab::pass16<false>(v, l, tw);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) X[col * kZLD + 8 * k1 + l] = v[k1];
    }
    __syncthreads();
    {
        cd a[8], bb[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = X[col * kZLD + 8 * l + n2];
            bb[n2] = X[col * kZLD + 8 * (l + 8) + n2];
        }
        slab::dft8<false>(a);
        slab::dft8<false>(bb);
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            X[col * kZLD + l + 16 * k2] = a[k2];
            X[col * kZLD + l + 8 + 16 * k2] = bb[k2];
        }
    }
    __syncthreads();
    for (int q = t; q < slab::N * kZR; q += kZThreads) {
        const int kz = q / kZR, qr = q - kz * kZR;
        const int r = r0 + qr;
        const int ky = r / slab::NH, kx = r - ky * slab::NH;
        hipfftDoubleComplex v6[6];
        for (int cc = 0; cc < 6; ++cc) {
            const cd x = X[(cc * kZR + qr) * kZLD + kz];
            v6[cc].x = x.re;
            v6[cc].y = x.im;
        }
        if (r == 0 && kz == 0)
            gamma_zero(v6, f, lam0, mu0, bc);
        else
            gamma_point(v6, f, kx, ky, kz, lam0, mu0);
        for (int cc = 0; cc < 6; ++cc) X[(cc * kZR + qr) * kZLD + kz] = {v6[cc].x, v6[cc].y};
    }
    __syncthreads();
    {
        cd v[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) v[n1] = X[col * kZLD + 8 * n1 + l];
        slab::pass16<true>(v, l, tw);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) X[col * kZLD + 8 * k1 + l] = v[k1];
    }
    __syncthreads();
    {
        cd a[8], bb[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = X[col * kZLD + 8 * l + n2];
            bb[n2] = X[col * kZLD + 8 * (l + 8) + n2];
        }
        slab::dft8<true>(a);
        slab::dft8<true>(bb);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            base[(int64_t)(l + 16 * k2) * 6 * P] = a[k2];
            base[(int64_t)(l + 8 + 16 * k2) * 6 * P] = bb[k2];
        }
    }
}

// The same for grids with nz = 150 (zfft150.hpp) on component-major spectra
// (value c of frequency (kx, ky, kz) at c cs + kz zs + r, r = ky nxh + kx)
// between 2-D in-plane hipFFT transforms: kZ150R frequencies r per
// work-group, 16 lanes per column (ten of them in the radix-15 pass,
// fifteen in the radix-10 pass).
constexpr int kZ150R = 8;  // eight frequencies: 128-byte segments per (z, c)
constexpr int kZ150Threads = 6 * kZ150R * 16;
constexpr int kZ150LD = z150::N + 1;
__global__ __launch_bounds__(kZ150Threads) void z150_gamma_kernel(hipfftDoubleComplex *spec,
                                                                  MsField f, double lam0,
                                                                  double mu0, MacroBC bc,
                                                                  int64_t cs, int64_t zs) {
    using slab::cd;
    __shared__ cd X[6 * kZ150R * kZ150LD];
    __shared__ cd tw[z150::N];
    z150::init_twiddles(tw);
    const int grp = xcd_group((int)blockIdx.x, (int)gridDim.x);
    const int nxh = f.nx / 2 + 1;
    const int r0 = grp * kZ150R;
    const int t = threadIdx.x;
    const int rr = t & (kZ150R - 1), l = (t / kZ150R) & 15, c = t / (kZ150R * 16);
    const int col = c * kZ150R + rr;
    cd *base = reinterpret_cast<cd *>(spec) + (int64_t)c * cs + r0 + rr;  // + z zs
    cd *Xc = X + col * kZ150LD;
    __syncthreads();
    {
        cd v[15];
        if (l < 10) {
#pragma unroll
            for (int n1 = 0; n1 < 15; ++n1) v[n1] = base[(int64_t)(10 * n1 + l) * zs];
            z150::pass15<false>(v, l, tw);
#pragma unroll
            for (int k1 = 0; k1 < 15; ++k1) Xc[10 * k1 + l] = v[k1];
        }
    }
    __syncthreads();
    {
        cd v[10];
        if (l < 15) {
#pragma unroll
            for (int n2 = 0; n2 < 10; ++n2) v[n2] = Xc[10 * l + n2];
            z150::dft10<false>(v, tw);
        }
        __syncthreads();
        if (l < 15) {
#pragma unroll
            for (int k2 = 0; k2 < 10; ++k2) Xc[l + 15 * k2] = v[k2];
        }
    }
    __syncthreads();
    for (int q = t; q < z150::N * kZ150R; q += kZ150Threads) {
        const int kz = q / kZ150R, qr = q - kz * kZ150R;
        const int r = r0 + qr;
        const int ky = r / nxh, kx = r - ky * nxh;
        hipfftDoubleComplex v6[6];
        for (int cc = 0; cc < 6; ++cc) {
            const cd x = X[(cc * kZ150R + qr) * kZ150LD + kz];
            v6[cc].x = x.re;
            v6[cc].y = x.im;
        }
        if (r == 0 && kz == 0)
            gamma_zero(v6, f, lam0, mu0, bc);
        else
            gamma_point(v6, f, kx, ky, kz, lam0, mu0);
        for (int cc = 0; cc < 6; ++cc) X[(cc * kZ150R + qr) * kZ150LD + kz] = {v6[cc].x, v6[cc].y};
    }
    __syncthreads();
    {
        cd v[15];
        if (l < 10) {
#pragma unroll
            for (int n1 = 0; n1 < 15; ++n1) v[n1] = Xc[10 * n1 + l];
            z150::pass15<true>(v, l, tw);
        }
        __syncthreads();
        if (l < 10) {
#pragma unroll
            for (int k1 = 0; k1 < 15; ++k1) Xc[10 * k1 + l] = v[k1];
        }
    }
    __syncthreads();
    {
        cd v[10];
        if (l < 15) {
#pragma unroll
            for (int n2 = 0; n2 < 10; ++n2) v[n2] = Xc[10 * l + n2];
            z150::dft10<true>(v, tw);
#pragma unroll
            for (int k2 = 0; k2 < 10; ++k2) base[(int64_t)(l + 15 * k2) * zs] = v[k2];
        }
    }
}

// In-plane transforms of 128 x 128 planes (slab_fft.hpp), one work-group
// per compute unit looping over the 6 nz planes (component-major real
// fields, plane-major spectra: plane (c, z) at spec + (6 z + c) 128 * 65).
__global__ __launch_bounds__(slab::kThreads) void xy_forward_kernel(const double *tau,
                                                                    slab::cd *spec, int nz) {
    // the packed plane (R x LD) and, at the end of each plane, its half
    // spectrum in memory order (N x NH)
    __shared__ slab::cd L[slab::N * slab::NH > slab::R * slab::LD ? slab::N * slab::NH
                                                                   : slab::R * slab::LD];
    __shared__ slab::cd tw[slab::N];
    slab::init_twiddles(tw);
    __syncthreads();
    const int64_t plane = (int64_t)slab::N * slab::N, P = (int64_t)slab::N * slab::NH;
    // each plane's rows are loaded while the previous plane is transformed
    slab::cd v[16];
    if ((int)blockIdx.x < 6 * nz) slab::load_rows(tau + (int64_t)blockIdx.x * plane, v);
    for (int p = blockIdx.x; p < 6 * nz; p += gridDim.x) {
        const int c = p / nz, z = p - c * nz;
        const int pn = p + (int)gridDim.x;
        slab::forward_plane(v, pn < 6 * nz ? tau + pn * plane : nullptr,
                            spec + ((int64_t)z * 6 + c) * P, L, tw);
    }
}

// The inverse in-plane transforms followed by the strain update
// eps <- raw / n with the per-block partial sums of the tensor-norm square
// of the change (partial[blockIdx.x], fixed order).
__global__ __launch_bounds__(slab::kThreads) void xy_inverse_update_kernel(
    const slab::cd *spec, double *eps, int nz, double inv_n, double *partial) {
    // the packed plane (R x LD) and, at the start of each plane, its half
    // spectrum in memory order (N x NH)
    __shared__ slab::cd L[slab::N * slab::NH > slab::R * slab::LD ? slab::N * slab::NH
                                                                   : slab::R * slab::LD];
    __shared__ slab::cd tw[slab::N];
    __shared__ double red[slab::kThreads];
    slab::init_twiddles(tw);
    __syncthreads();
    const int64_t plane = (int64_t)slab::N * slab::N, P = (int64_t)slab::N * slab::NH;
    double acc = 0.0;
    for (int p = blockIdx.x; p < 6 * nz; p += gridDim.x) {
        const int c = p / nz, z = p - c * nz;
        slab::inverse_plane_update(spec + ((int64_t)z * 6 + c) * P, eps + p * plane, inv_n,
                                   c < 3 ? 1.0 : 0.5, acc, L, tw);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = slab::kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
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
// fold (optional, the step's failure counters): fold[0] += fold[1],
// fold[1] = 0, by one thread (stream order makes it safe).
__global__ __launch_bounds__(kRedBlock) void finish_kernel(const double *partial, int m,
                                                           double *out,
                                                           uint64_t *fold = nullptr) {
    if (fold && blockIdx.x == 0 && threadIdx.x == 0) {
        fold[0] += fold[1];
        fold[1] = 0;
    }
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

// per-block min and max of the Lame constants of the isotropic parts of a
// tangent field [36][n] (row-major 6x6 per point): partial[4][gridDim.x] =
// min lambda, max lambda, min mu, max mu (NaN entries are skipped)
__global__ __launch_bounds__(kRedBlock) void iso_minmax_kernel(const double *C, int64_t n,
                                                               double *partial) {
    __shared__ double red[4][kRedBlock];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock) {
        double k3 = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) k3 += C[(6 * r + c) * n + i];
        k3 *= 1.0 / 3.0;  // 3 K
        const double isym = C[0 * n + i] + C[7 * n + i] + C[14 * n + i] +
                            2.0 * (C[21 * n + i] + C[28 * n + i] + C[35 * n + i]);
        const double mu = (isym - k3) / 10.0;
        const double lam = (k3 - 2.0 * mu) / 3.0;
        v[0] = fmin(v[0], lam);
        v[1] = fmax(v[1], lam);
        v[2] = fmin(v[2], mu);
        v[3] = fmax(v[3], mu);
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k)
                red[k][threadIdx.x] = (k & 1) ? fmax(red[k][threadIdx.x], red[k][threadIdx.x + w])
                                              : fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) partial[k * gridDim.x + blockIdx.x] = red[k][0];
}

// min (even rows) or max (odd rows) of m partials per row
__global__ __launch_bounds__(kRedBlock) void finish_minmax_kernel(const double *partial, int m,
                                                                  double *out) {
    __shared__ double red[kRedBlock];
    const bool mx = blockIdx.x & 1;
    double s = mx ? -INFINITY : INFINITY;
    for (int b = threadIdx.x; b < m; b += kRedBlock) {
        const double x = partial[blockIdx.x * m + b];
        s = mx ? fmax(s, x) : fmin(s, x);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = mx ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                  : fmin(red[threadIdx.x], red[threadIdx.x + w]);
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
    // grids with nx = ny = 128: in-plane transforms by the slab kernels,
    // the transforms along z (plane-major spectrum) with Gamma0 between them
    // by z_gamma_kernel where nz = 128 too (zfused), else by zfft
    bool slab, zfused;
    int slab_grid;
    hipfftHandle zfft;
    // grids with nz = 150 (other in-plane sizes): 2-D hipFFT transforms over
    // (y, x) and z150_gamma_kernel along z
    bool z150;
    hipfftHandle fwd2, inv2;
    double *sig;   // [6][n] stress / polarization / raw inverse FFT output
    double *dlt;   // [6][n] increments a_{n+1} - a_n of the last sweep: the next
                   // sweep's Newton solves start there (warm start)
    hipfftDoubleComplex *spec;  // [6][nh]
    double *partial;            // [6 * kRedBlocks]
    double *scal;               // [16] reduced scalars; [8..13] the macro strain
    uint64_t *fails;            // device [2]: point solves of the current step that failed,
                                // and those of a sweep started ahead of a convergence test
    hipEvent_t ev_scal;         // the reduced scalars have reached the host
    uint64_t *host_fails;       // pinned
    uint64_t last_fails;        // of the last completed step
    double *host_scal;          // pinned [16]
    // the fixed-point iteration's scalars (norm at [0], macro strain at
    // [8..13]), written by the kernels straight into pinned host memory
    double *iter_host, *iter_dev;
    // reverse step work space, allocated on first use
    double *tan;                // [36][n] consistent tangent at the converged strain
    double *lam;                // [6][n] adjoint field
    double *rhs;                // [6][n] right-hand side / scratch
    double *gs;                 // [6][n] stress cotangent
};

static int32_t ms_check_opts(const automat_ms_options *o) {
    if (!o) return AUTOMAT_EINVAL;
    if (o->max_iter < 1 || o->newton_max_iter < 1) return AUTOMAT_EINVAL;
    if (o->ref_update != 0 && o->ref_update != 1) return AUTOMAT_EINVAL;
    if (o->warm_start != 0 && o->warm_start != 1) return AUTOMAT_EINVAL;
    if (o->reserved != 0) return AUTOMAT_EINVAL;
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
              (!opts->warm_start ||
               (hipMalloc(&m->dlt, nb) == hipSuccess && hipMemset(m->dlt, 0, nb) == hipSuccess)) &&
              hipMalloc(&m->spec, nc) == hipSuccess &&
              hipMalloc(&m->partial, 6 * kRedBlocks * sizeof(double)) == hipSuccess &&
              hipMalloc(&m->scal, 16 * sizeof(double)) == hipSuccess &&
              hipHostMalloc(&m->host_scal, 16 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&m->iter_host, 16 * sizeof(double),
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostGetDevicePointer(reinterpret_cast<void **>(&m->iter_dev), m->iter_host, 0) ==
                  hipSuccess &&
              hipMalloc(&m->fails, 2 * sizeof(uint64_t)) == hipSuccess &&
              hipEventCreateWithFlags(&m->ev_scal, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc(&m->host_fails, sizeof(uint64_t), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipfftPlanMany(&m->fwd, 3, dims, dims, 1, (int)m->f.n, dims_c, 1, (int)m->f.nh,
                              HIPFFT_D2Z, 6) == HIPFFT_SUCCESS;
    ok = ok && hipfftPlanMany(&m->inv, 3, dims, dims_c, 1, (int)m->f.nh, dims, 1, (int)m->f.n,
                              HIPFFT_Z2D, 6) == HIPFFT_SUCCESS;
    m->slab = nx == slab::N && ny == slab::N;
    if (ok && m->slab) {
        const int planes = (int)(ny * (nx / 2 + 1)) * 6;  // columns along z, unit distance
        int len[1] = {nz};
        int cus = 0, dev = 0;
        ok = hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
             cus > 0;
        const int work = 6 * nz;
        m->slab_grid = work < cus ? work : cus;
        if (m->slab_grid > kRedBlocks) m->slab_grid = kRedBlocks;
        m->zfused = nz == slab::N;
        ok = ok && (m->zfused || hipfftPlanMany(&m->zfft, 1, len, len, planes, 1, len, planes, 1,
                                                HIPFFT_Z2Z, planes) == HIPFFT_SUCCESS);
    }
    m->z150 = !m->slab && nz == z150::N && (int64_t)ny * (nx / 2 + 1) % kZ150R == 0;
    if (ok && m->z150) {
        int d2[2] = {ny, nx}, d2c[2] = {ny, nx / 2 + 1};
        const int pr = ny * nx, pc = ny * (nx / 2 + 1);
        ok = hipfftPlanMany(&m->fwd2, 2, d2, d2, 1, pr, d2c, 1, pc, HIPFFT_D2Z, 6 * nz) ==
                 HIPFFT_SUCCESS &&
             hipfftPlanMany(&m->inv2, 2, d2, d2c, 1, pc, d2, 1, pr, HIPFFT_Z2D, 6 * nz) ==
                 HIPFFT_SUCCESS;
    }
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
    if (m->zfft) (void)hipfftDestroy(m->zfft);
    if (m->fwd2) (void)hipfftDestroy(m->fwd2);
    if (m->inv2) (void)hipfftDestroy(m->inv2);
    if (m->sig) (void)hipFree(m->sig);
    if (m->dlt) (void)hipFree(m->dlt);
    if (m->spec) (void)hipFree(m->spec);
    if (m->partial) (void)hipFree(m->partial);
    if (m->scal) (void)hipFree(m->scal);
    if (m->host_scal) (void)hipHostFree(m->host_scal);
    if (m->iter_host) (void)hipHostFree(m->iter_host);
    if (m->fails) (void)hipFree(m->fails);
    if (m->ev_scal) (void)hipEventDestroy(m->ev_scal);
    if (m->host_fails) (void)hipHostFree(m->host_fails);
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

// the warm-start buffer, or null without warm starts
static double *warm(automat_ms *m) { return m->opts.warm_start ? m->dlt : nullptr; }

static int32_t ensure_buffer(double **p, size_t bytes) {
    if (*p) return AUTOMAT_OK;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return AUTOMAT_ENOMEM;
    }
    return AUTOMAT_OK;
}

static int32_t read_scalars(automat_ms *m, const double *scal, int count, hipStream_t s) {
    if (hipMemcpyAsync(m->host_scal, scal, count * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

// C0 from the tangent field at the current strain (a_n fixed): the means of
// the extreme Lame constants of the isotropic parts
static int32_t update_reference(automat_ms *m, const uint8_t *phase, double h, const double *eps,
                                const double *a, hipStream_t s, int rb) {
    const int64_t n = m->f.n;
    int32_t rc = ensure_buffer(&m->tan, (size_t)n * 36 * sizeof(double));
    if (rc) return rc;
    rc = evaluate_warm(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                       m->opts.newton_max_iter, m->sig, nullptr, m->tan, warm(m), nullptr,
                       m->fails, s);
    if (rc) return rc;
    hipLaunchKernelGGL(iso_minmax_kernel, dim3(rb), dim3(kRedBlock), 0, s, m->tan, n, m->partial);
    hipLaunchKernelGGL(finish_minmax_kernel, dim3(4), dim3(kRedBlock), 0, s, m->partial, rb,
                       m->scal);
    rc = read_scalars(m, m->scal, 4, s);
    if (rc) return rc;
    const double lam0 = 0.5 * (m->host_scal[0] + m->host_scal[1]);
    const double mu0 = 0.5 * (m->host_scal[2] + m->host_scal[3]);
    if (!std::isfinite(lam0) || !(mu0 > 0.0) || !(lam0 + 2.0 * mu0 / 3.0 > 0.0))
        return AUTOMAT_EINVAL;
    m->lam0 = lam0;
    m->mu0 = mu0;
    return AUTOMAT_OK;
}

// Work space of one load step: the polarization / inverse-transform field,
// its half spectrum, the reduction partials, the reduced scalars and the
// failed-solve counter.
struct MsWork {
    double *sig;                // [6][n]
    hipfftDoubleComplex *spec;  // [6][nh]
    double *partial;            // [6 * kRedBlocks]
    double *scal;               // [16]
    uint64_t *fails;            // [2]
};

__global__ void zero_u64_kernel(uint64_t *p) { p[0] = p[1] = 0; }

static int32_t ms_step_impl(automat_ms *m, const MsWork &w, const uint8_t *phase,
                            const double *E_macro, const double *S_macro, uint32_t stress_mask,
                            double h, double *eps, double *a, double *sigma_out,
                            double *sigma_mean, double *E_reached, int32_t *iters,
                            double *residual, void *stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = m->f.n;
    const int tb = 256;
    const int gb = (int)((n + tb - 1) / tb);
    if (hipfftSetStream(m->fwd, s) != HIPFFT_SUCCESS || hipfftSetStream(m->inv, s) != HIPFFT_SUCCESS ||
        (m->zfft && hipfftSetStream(m->zfft, s) != HIPFFT_SUCCESS) ||
        (m->fwd2 && (hipfftSetStream(m->fwd2, s) != HIPFFT_SUCCESS ||
                     hipfftSetStream(m->inv2, s) != HIPFFT_SUCCESS)))
        return AUTOMAT_EHIP;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, w.fails);
    MacroBC bc;
    for (int c = 0; c < 6; ++c) {
        bc.E[c] = (stress_mask >> c & 1u) ? 0.0 : E_macro[c];
        bc.S[c] = S_macro ? S_macro[c] : 0.0;
    }
    bc.mask = stress_mask;
    bc.Eout = m->iter_dev + 8;
    // initial guess: previous strain field shifted by the prescribed strain
    // increments and, on stress-controlled components, the increments that
    // keep the reference medium's stress there unchanged
    double dE[6], d[6];  // d: prescribed increments, zero on the stress-controlled set
    for (int c = 0; c < 6; ++c) d[c] = (stress_mask >> c & 1u) ? 0.0 : E_macro[c] - m->E_prev[c];
    if (stress_mask) {
        const double zero[6] = {0, 0, 0, 0, 0, 0};
        mixed_solve(m->lam0, m->mu0, stress_mask, d, zero, dE);
    } else {
        for (int c = 0; c < 6; ++c) dE[c] = d[c];
    }
    hipLaunchKernelGGL(shift_kernel, dim3(gb), dim3(tb), 0, s, eps, n, dE[0], dE[1], dE[2], dE[3],
                       dE[4], dE[5]);
    double Ecur[6];
    for (int c = 0; c < 6; ++c) Ecur[c] = m->E_prev[c] + dE[c];
    const int nhb = (int)((m->f.nh + tb - 1) / tb);
    const int rb = (int)((n + kRedBlock - 1) / kRedBlock) < kRedBlocks
                       ? (int)((n + kRedBlock - 1) / kRedBlock)
                       : kRedBlocks;
    int32_t rc = AUTOMAT_OK;
    if (m->opts.ref_update) {
        rc = update_reference(m, phase, h, eps, a, s, rb);
        if (rc) return rc;
    }
    int it = 0;
    double err = 0.0;
    // While the host waits for an iteration's convergence test, the next
    // iteration's sweep (which reads only the updated strain) already runs;
    // its failures go to the second counter and are folded in when it is
    // used, and a converged step discards it.
    bool ahead = false;
    for (it = 1; it <= m->opts.max_iter; ++it) {
        const bool swept = ahead;
        ahead = false;
        // material sweep writing the polarization tau = sigma - C0 eps
        if (!swept) {
            rc = evaluate_polarized(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                                    m->opts.newton_max_iter, m->lam0, m->mu0, w.sig, warm(m),
                                    w.fails, stream);
            if (rc) return rc;
        }
        uint64_t *fold = swept ? w.fails : nullptr;
        if (m->slab) {
            const int64_t P = (int64_t)m->f.ny * (m->f.nx / 2 + 1);
            slab::cd *sp = reinterpret_cast<slab::cd *>(w.spec);
            hipLaunchKernelGGL(xy_forward_kernel, dim3(m->slab_grid), dim3(slab::kThreads), 0, s,
                               w.sig, sp, m->f.nz);
            if (m->zfused) {
                hipLaunchKernelGGL(z_gamma_kernel, dim3((int)(P / kZR)), dim3(kZThreads), 0, s, sp,
                                   m->f, m->lam0, m->mu0, bc);
            } else {
                if (hipfftExecZ2Z(m->zfft, w.spec, w.spec, HIPFFT_FORWARD) != HIPFFT_SUCCESS)
                    return AUTOMAT_EHIP;
                hipLaunchKernelGGL(gamma_kernel, dim3(nhb), dim3(tb), 0, s, w.spec, m->f, m->lam0,
                                   m->mu0, bc, P, 6 * P);
                if (hipfftExecZ2Z(m->zfft, w.spec, w.spec, HIPFFT_BACKWARD) != HIPFFT_SUCCESS)
                    return AUTOMAT_EHIP;
            }
            hipLaunchKernelGGL(xy_inverse_update_kernel, dim3(m->slab_grid), dim3(slab::kThreads),
                               0, s, sp, eps, m->f.nz, 1.0 / (double)n, w.partial);
            hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kRedBlock), 0, s, w.partial,
                               m->slab_grid, m->iter_dev, fold);
        } else {
            const int64_t P = (int64_t)m->f.ny * (m->f.nx / 2 + 1);
            if (m->z150) {
                if (hipfftExecD2Z(m->fwd2, w.sig, w.spec) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
                hipLaunchKernelGGL(z150_gamma_kernel, dim3((int)(P / kZ150R)), dim3(kZ150Threads), 0,
                                   s, w.spec, m->f, m->lam0, m->mu0, bc, m->f.nh, P);
                if (hipfftExecZ2D(m->inv2, w.spec, w.sig) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
            } else {
                if (hipfftExecD2Z(m->fwd, w.sig, w.spec) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
                hipLaunchKernelGGL(gamma_kernel, dim3(nhb), dim3(tb), 0, s, w.spec, m->f, m->lam0,
                                   m->mu0, bc, m->f.nh, P);
                if (hipfftExecZ2D(m->inv, w.spec, w.sig) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
            }
            hipLaunchKernelGGL(update_kernel, dim3(rb), dim3(kRedBlock), 0, s, eps, w.sig, n,
                               w.partial);
            hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kRedBlock), 0, s, w.partial, rb,
                               m->iter_dev, fold);
        }
        if (!m->opts.fixed_iter || it == m->opts.max_iter) {
            // the scalars are in host memory once this iteration's kernels are done
            if (hipEventRecord(m->ev_scal, s) != hipSuccess) return AUTOMAT_EHIP;
            if (!m->opts.fixed_iter && it < m->opts.max_iter) {
                rc = evaluate_polarized(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                                        m->opts.newton_max_iter, m->lam0, m->mu0, w.sig, warm(m),
                                        w.fails + 1, stream);
                if (rc) return rc;
                ahead = true;
            }
            if (hipEventSynchronize(m->ev_scal) != hipSuccess) return AUTOMAT_EHIP;
            volatile const double *hs = m->iter_host;
            for (int c = 0; c < 6; ++c) Ecur[c] = hs[8 + c];
            err = sqrt(hs[0] / (double)n) / fmax(tensor_norm(Ecur), 1e-300);
            if (!m->opts.fixed_iter && err <= m->opts.tol) break;
        }
    }
    if (it > m->opts.max_iter) it = m->opts.max_iter;
    // commit: sweep at the converged strain, a_n <- a_{n+1}
    double *sig = sigma_out ? sigma_out : w.sig;
    rc = evaluate_warm(n, eps, a, phase, &m->params, h, m->opts.newton_tol,
                       m->opts.newton_max_iter, sig, a, nullptr, warm(m), warm(m), w.fails,
                       stream);
    if (rc) return rc;
    if (sigma_mean) {
        hipLaunchKernelGGL(mean6_kernel, dim3(rb), dim3(kRedBlock), 0, s, sig, n, w.partial);
        hipLaunchKernelGGL(finish_kernel, dim3(6), dim3(kRedBlock), 0, s, w.partial, rb, w.scal);
        rc = read_scalars(m, w.scal, 6, s);
        if (rc) return rc;
        for (int c = 0; c < 6; ++c) sigma_mean[c] = m->host_scal[c] / (double)n;
    }
    if (hipMemcpyAsync(m->host_fails, w.fails, sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AUTOMAT_EHIP;
    m->last_fails = *m->host_fails;
    for (int c = 0; c < 6; ++c) {
        m->E_prev[c] = Ecur[c];
        if (E_reached) E_reached[c] = Ecur[c];
    }
    if (iters) *iters = it;
    if (residual) *residual = err;
    if (hipGetLastError() != hipSuccess) return AUTOMAT_EHIP;
    return AUTOMAT_OK;
}

extern "C" int32_t automat_ms_step_mixed(automat_ms *m, const uint8_t *phase,
                                         const double *E_macro, const double *S_macro,
                                         uint32_t stress_mask, double h, double *eps, double *a,
                                         double *sigma_out, double *sigma_mean,
                                         double *E_reached, int32_t *iters, double *residual,
                                         void *stream) {
    if (!m || !phase || !E_macro || !eps || !a) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0) || stress_mask > 63u) return AUTOMAT_EINVAL;
    const MsWork w{m->sig, m->spec, m->partial, m->scal, m->fails};
    return ms_step_impl(m, w, phase, E_macro, S_macro, stress_mask, h, eps, a, sigma_out,
                        sigma_mean, E_reached, iters, residual, stream);
}

extern "C" int32_t automat_ms_step(automat_ms *m, const uint8_t *phase, const double *E_macro,
                                   double h, double *eps, double *a, double *sigma_out,
                                   double *sigma_mean, int32_t *iters, double *residual,
                                   void *stream) {
    return automat_ms_step_mixed(m, phase, E_macro, nullptr, 0u, h, eps, a, sigma_out, sigma_mean,
                                 nullptr, iters, residual, stream);
}

// --------------------------------------------------------------------------
// The load step without allocation: the step's work space lives in a
// file-scope device array (one copy per device, held until the process
// ends) instead of the handle's buffers. Host code never passes the array's
// name to a kernel or copy: its device address is taken once per device
// with hipGetSymbolAddress and kept.
// --------------------------------------------------------------------------

constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[64];
static bool g_scratch_init[64];

static int32_t scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return AUTOMAT_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_init[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return AUTOMAT_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
        g_scratch_init[dev] = true;
    }
    *out = g_scratch_ptr[dev];
    return AUTOMAT_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" int32_t automat_ms_step_noalloc(automat_ms *m, const uint8_t *phase,
                                           const double *E_macro, double h, double *eps,
                                           double *a, double *sigma_out, double *sigma_mean,
                                           int32_t *iters, double *residual, void *stream) {
    if (!m || !phase || !E_macro || !eps || !a) return AUTOMAT_EINVAL;
    if (!std::isfinite(h) || !(h > 0.0)) return AUTOMAT_EINVAL;
    if (m->opts.ref_update) return AUTOMAT_EINVAL;  // its tangent field is not in the work space
    const size_t b_sig = align256((size_t)m->f.n * 6 * sizeof(double));
    const size_t b_spec = align256((size_t)m->f.nh * 6 * sizeof(hipfftDoubleComplex));
    const size_t b_part = align256((size_t)6 * kRedBlocks * sizeof(double));
    const size_t b_scal = align256(16 * sizeof(double));
    if (b_sig + b_spec + b_part + b_scal + 256 > kScratchBytes) return AUTOMAT_EINVAL;
    void *base = nullptr;
    const int32_t rc = scratch_address(&base);
    if (rc) return rc;
    char *p = static_cast<char *>(base);
    MsWork w;
    w.sig = reinterpret_cast<double *>(p);
    w.spec = reinterpret_cast<hipfftDoubleComplex *>(p + b_sig);
    w.partial = reinterpret_cast<double *>(p + b_sig + b_spec);
    w.scal = reinterpret_cast<double *>(p + b_sig + b_spec + b_part);
    w.fails = reinterpret_cast<uint64_t *>(p + b_sig + b_spec + b_part + b_scal);
    return ms_step_impl(m, w, phase, E_macro, nullptr, 0u, h, eps, a, sigma_out, sigma_mean,
                        nullptr, iters, residual, stream);
}

extern "C" int32_t automat_ms_newton_failures(const automat_ms *m, uint64_t *count) {
    if (!m || !count) return AUTOMAT_EINVAL;
    *count = m->last_fails;
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
    MacroBC bc;
    std::memset(&bc, 0, sizeof bc);  // zero mean: eps^(0) = 0
    if (hipMemcpyAsync(m->sig, x, (size_t)m->f.n * 6 * sizeof(double), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        return AUTOMAT_EHIP;
    if (hipfftExecD2Z(m->fwd, m->sig, m->spec) != HIPFFT_SUCCESS) return AUTOMAT_EHIP;
    hipLaunchKernelGGL(gamma_kernel, dim3(nhb), dim3(tb), 0, s, m->spec, m->f, m->lam0, m->mu0,
                       bc, m->f.nh, (int64_t)m->f.ny * (m->f.nx / 2 + 1));
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
    if (ensure_buffer(&m->tan, 6 * fb) || ensure_buffer(&m->lam, fb) ||
        ensure_buffer(&m->rhs, fb) || ensure_buffer(&m->gs, fb))
        return AUTOMAT_ENOMEM;
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
