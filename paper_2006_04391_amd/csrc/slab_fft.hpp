// slab_fft.hpp -- the in-plane (x, y) part of the basic scheme's transforms
// for grids with nx = ny = 128, one z plane of one component per pass of a
// work-group, entirely in LDS.
//
// Forward: a real 128 x 128 plane r[y][x] becomes its half spectrum
// S[ky][kx], kx = 0 .. 64 (the layout of a real-to-complex transform).
// Rows are transformed two at a time as one complex sequence
// z = r[2y'] + i r[2y'+1] (64 complex rows of 128); the two real rows'
// spectra separate as A[k] = (Z[k] + conj Z[-k]) / 2 and
// B[k] = (Z[k] - conj Z[-k]) / (2i). The columns kx = 1 .. 63 are then
// complex sequences along y; the two real-valued columns kx = 0 and 64 are
// transformed together as one complex column c0 + i c64 and separated the
// same way. Every length-128 transform is a radix-16 pass (over n1 with
// n = 8 n1 + n2, then the twiddle exp(-2 pi i n2 k1 / 128)) followed by a
// radix-8 pass (over n2, k = k1 + 16 k2), both in registers, with LDS
// between them.
//
// Inverse: the reverse steps (columns first, then rows, two real rows per
// complex row; the kx = 0 and 64 columns again as one complex column),
// unnormalised like the forward, followed in the same kernel by the strain
// update of the fixed-point iteration: eps' = raw / n, the tensor-norm
// square of eps' - eps summed per work-group in a fixed order, eps <- eps'.
//
// The half spectrum moves between memory and LDS in one contiguous pass per
// plane (its rows of 65 complex values start mid-line, so column-wise
// accesses would touch each line more than once).
//
// LDS holds the packed plane as 64 rows of 128 complex values (pitch 129).
// After the row pass, column j (0 .. 63) keeps its 128 values in the cells
// (q, j) and (q, 128 - j) of rows q = 0 .. 63 (column 0: (q, 0) and (q, 64)),
// so the 64 columns own disjoint cells and the plane is transformed in
// place.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace automat {
namespace slab {

constexpr int N = 128;          // in-plane extent
constexpr int NH = N / 2 + 1;   // half-spectrum row length
constexpr int R = N / 2;        // packed rows (and columns)
constexpr int LD = N + 1;       // LDS pitch, in complex values
constexpr int kThreads = 512;   // 8 lanes per packed row / column

struct cd {
    double re, im;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a times exp(-i pi / 2) (forward) or exp(+i pi / 2) (inverse)
template <bool INV>
__device__ __forceinline__ cd rot4(cd a) {
    return INV ? cd{-a.im, a.re} : cd{a.im, -a.re};
}
// a times w (forward) or conj(w) (inverse), w = (c, s) an exp(-i theta)
template <bool INV>
__device__ __forceinline__ cd twid(cd a, double c, double s) {
    return INV ? cd{a.re * c + a.im * s, a.im * c - a.re * s}
               : cd{a.re * c - a.im * s, a.im * c + a.re * s};
}

// Discrete Fourier transforms of length 4, 8 and 16 in natural order,
// X[k] = sum_n x[n] exp(-+2 pi i n k / L), by even/odd splitting.
template <bool INV>
__device__ __forceinline__ void dft4(cd &a0, cd &a1, cd &a2, cd &a3) {
    const cd s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = rot4<INV>(a1 - a3);
    a0 = s02 + s13;
    a2 = s02 - s13;
    a1 = d02 + d13;
    a3 = d02 - d13;
}

constexpr double kR2 = 0.70710678118654752440;   // cos(pi / 4)
constexpr double kC8 = 0.92387953251128675613;   // cos(pi / 8)
constexpr double kS8 = 0.38268343236508977173;   // sin(pi / 8)

template <bool INV>
__device__ __forceinline__ void dft8(cd *v) {
    cd e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cd o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    // twiddles exp(-2 pi i k / 8), k = 1, 2, 3: (r, -r), (0, -1), (-r, -r)
    o1 = twid<INV>(o1, kR2, -kR2);
    o2 = rot4<INV>(o2);
    o3 = twid<INV>(o3, -kR2, -kR2);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
}

template <bool INV>
__device__ __forceinline__ void dft16(cd *v) {
    cd e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        e[k] = v[2 * k];
        o[k] = v[2 * k + 1];
    }
    dft8<INV>(e);
    dft8<INV>(o);
    // exp(-2 pi i k / 16) = (cos(k pi / 8), -sin(k pi / 8))
    o[1] = twid<INV>(o[1], kC8, -kS8);
    o[2] = twid<INV>(o[2], kR2, -kR2);
    o[3] = twid<INV>(o[3], kS8, -kC8);
    o[4] = rot4<INV>(o[4]);
    o[5] = twid<INV>(o[5], -kS8, -kC8);
    o[6] = twid<INV>(o[6], -kR2, -kR2);
    o[7] = twid<INV>(o[7], -kC8, -kS8);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = e[k] + o[k];
        v[k + 8] = e[k] - o[k];
    }
}

// LDS cell of value q (0 .. 127) of packed column j after the row pass
__device__ __forceinline__ int cell(int j, int q) {
    const int col = q < R ? j : (j ? N - j : R);
    return (q & (R - 1)) * LD + col;
}

// the radix-16 pass of one length-128 transform: v[n1] = x[8 n1 + n2] in,
// twiddled partial transforms [k1] out
template <bool INV>
__device__ __forceinline__ void pass16(cd *v, int n2, const cd *tw) {
    dft16<INV>(v);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) {
        const cd w = tw[n2 * k1];
        v[k1] = twid<INV>(v[k1], w.re, w.im);
    }
}

// twiddle table exp(-2 pi i m / 128), m = 0 .. 127
__device__ __forceinline__ void init_twiddles(cd *tw) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s, c;
        sincospi((double)m / (double)R, &s, &c);
        tw[m] = {c, -s};
    }
}

// One forward plane: v holds its rows (load_rows), dst receives the half
// spectrum [128][65]; next (or null): the next plane, whose rows are loaded
// into v once this plane's rows are in LDS. L: LDS of max(R LD, N NH)
// complex values (the packed plane, then the half spectrum in memory order,
// stored to dst in one contiguous pass so that every line is written whole);
// tw: twiddles.
// The rows of a real plane as the radix-16 pass takes them: lane l of packed
// row g gets x = 8 n1 + l of rows 2g (real part) and 2g + 1 (imaginary part).
__device__ __forceinline__ void load_rows(const double *__restrict__ src, cd *v) {
    const int t = threadIdx.x;
    const int g = t >> 3, l = t & 7;
    const double *r0 = src + (2 * g) * N, *r1 = r0 + N;
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = {r0[8 * n1 + l], r1[8 * n1 + l]};
}

__device__ __forceinline__ void forward_plane(cd *v, const double *__restrict__ next,
                                              cd *__restrict__ dst, cd *L, const cd *tw) {
    const int t = threadIdx.x;
    const int g = t >> 3, l = t & 7;  // packed row or column g, lane l of its 8
    {
        // rows: radix-16 pass
        pass16<false>(v, l, tw);
        __syncthreads();  // the previous plane's last reads of L are done
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) L[g * LD + 8 * k1 + l] = v[k1];
        if (next) load_rows(next, v);
    }
    __syncthreads();
    {
        // rows: radix-8 pass, lane l takes k1 = l and l + 8
        cd a[8], b[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = L[g * LD + 8 * l + n2];
            b[n2] = L[g * LD + 8 * (l + 8) + n2];
        }
        dft8<false>(a);
        dft8<false>(b);
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            L[g * LD + l + 16 * k2] = a[k2];
            L[g * LD + l + 8 + 16 * k2] = b[k2];
        }
    }
    __syncthreads();
    {
        // columns: separate the two real rows of each packed row while
        // loading, radix-16 pass
        cd w[16];
        cd *v = w;
        const bool odd = l & 1;  // y = 8 n1 + l has the parity of l
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int yp = (8 * n1 + l) >> 1;
            if (g == 0) {
                const cd z0 = L[yp * LD], z64 = L[yp * LD + R];
                v[n1] = odd ? cd{z0.im, z64.im} : cd{z0.re, z64.re};
            } else {
                const cd a = L[yp * LD + g], b = L[yp * LD + N - g];
                v[n1] = odd ? cd{0.5 * (a.im + b.im), -0.5 * (a.re - b.re)}
                            : cd{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
            }
        }
        pass16<false>(v, l, tw);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) L[cell(g, 8 * k1 + l)] = v[k1];
    }
    __syncthreads();
    {
        // columns: radix-8 pass; columns 1 .. 63 go to memory, the packed
        // column 0 back to LDS in natural order
        cd a[8], b[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = L[cell(g, 8 * l + n2)];
            b[n2] = L[cell(g, 8 * (l + 8) + n2)];
        }
        dft8<false>(a);
        dft8<false>(b);
        __syncthreads();  // every column's cells are read
        // stage the half spectrum in LDS in its memory order [ky][kx]; the
        // packed column 0 goes to the kx = 0 slots for now
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            L[(l + 16 * k2) * NH + g] = a[k2];
            L[(l + 8 + 16 * k2) * NH + g] = b[k2];
        }
    }
    __syncthreads();
    {
        // separate the spectra of the real columns kx = 0 and 64
        cd q{0.0, 0.0}, qm{0.0, 0.0};
        if (t < N) {
            q = L[t * NH];
            qm = L[((N - t) & (N - 1)) * NH];
        }
        __syncthreads();
        if (t < N) {
            L[t * NH] = {0.5 * (q.re + qm.re), 0.5 * (q.im - qm.im)};
            L[t * NH + R] = {0.5 * (q.im + qm.im), -0.5 * (q.re - qm.re)};
        }
    }
    __syncthreads();
    // one contiguous store of the plane's half spectrum: whole lines
    for (int k = t; k < N * NH; k += kThreads) dst[k] = L[k];
}

// One inverse plane: src half spectrum [128][65], then the strain update of
// the real plane eps [128][128] with raw = the unnormalised inverse:
// eps' = raw * inv_n, acc += wgt * (eps' - eps)^2, eps <- eps'. L: LDS of
// max(R LD, N NH) complex values (the half spectrum in memory order, loaded
// in one contiguous pass so that every line is read whole, then the packed
// plane).
__device__ __forceinline__ void inverse_plane_update(const cd *__restrict__ src,
                                                     double *__restrict__ eps, double inv_n,
                                                     double wgt, double &acc, cd *L,
                                                     const cd *tw) {
    const int t = threadIdx.x;
    const int g = t >> 3, l = t & 7;
    {
        // the half spectrum into LDS in memory order (one contiguous load:
        // whole lines), then the columns (column 0 packs kx = 0 and 64):
        // radix-16 pass
        __syncthreads();  // the previous plane's last reads of L are done
        for (int k = t; k < N * NH; k += kThreads) L[k] = src[k];
        __syncthreads();
        cd v[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int ky = 8 * n1 + l;
            if (g) {
                v[n1] = L[ky * NH + g];
            } else {
                const cd s0 = L[ky * NH], s64 = L[ky * NH + R];
                v[n1] = {s0.re - s64.im, s0.im + s64.re};
            }
        }
        pass16<true>(v, l, tw);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) L[cell(g, 8 * k1 + l)] = v[k1];
    }
    __syncthreads();
    {
        // columns: radix-8 pass, results by y in the column's cells
        cd a[8], b[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = L[cell(g, 8 * l + n2)];
            b[n2] = L[cell(g, 8 * (l + 8) + n2)];
        }
        dft8<true>(a);
        dft8<true>(b);
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            L[cell(g, l + 16 * k2)] = a[k2];
            L[cell(g, l + 8 + 16 * k2)] = b[k2];
        }
    }
    __syncthreads();
    {
        // rows: pack real rows 2g and 2g + 1 as one complex row while
        // loading (Hermitian extension for kx > 64), radix-16 pass
        cd v[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int k = 8 * n1 + l;
            if (k == 0 || k == R) {
                const cd pe = L[cell(0, 2 * g)], po = L[cell(0, 2 * g + 1)];
                v[n1] = k == 0 ? cd{pe.re, po.re} : cd{pe.im, po.im};
            } else if (k < R) {
                const cd e = L[cell(k, 2 * g)], o = L[cell(k, 2 * g + 1)];
                v[n1] = {e.re - o.im, e.im + o.re};
            } else {
                const cd e = L[cell(N - k, 2 * g)], o = L[cell(N - k, 2 * g + 1)];
                v[n1] = {e.re + o.im, o.re - e.im};
            }
        }
        pass16<true>(v, l, tw);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) L[g * LD + 8 * k1 + l] = v[k1];
    }
    __syncthreads();
    {
        // rows: radix-8 pass, then the update of rows 2g and 2g + 1 (their
        // old strain is loaded first, in flight during the pass)
        double *e0 = eps + (2 * g) * N, *e1 = e0 + N;
        double old0[16], old1[16];
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                old0[2 * k2 + h] = e0[l + 8 * h + 16 * k2];
                old1[2 * k2 + h] = e1[l + 8 * h + 16 * k2];
            }
        cd a[8], b[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
            a[n2] = L[g * LD + 8 * l + n2];
            b[n2] = L[g * LD + 8 * (l + 8) + n2];
        }
        dft8<true>(a);
        dft8<true>(b);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const cd z = h ? b[k2] : a[k2];
                const int x = l + 8 * h + 16 * k2;
                const double n0 = z.re * inv_n, n1v = z.im * inv_n;
                const double d0 = n0 - old0[2 * k2 + h], d1 = n1v - old1[2 * k2 + h];
                acc += wgt * (d0 * d0 + d1 * d1);
                e0[x] = n0;
                e1[x] = n1v;
            }
        }
    }
}

}  // namespace slab
}  // namespace automat
