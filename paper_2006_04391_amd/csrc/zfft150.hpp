// zfft150.hpp -- length-150 transforms along z for the basic scheme's
// 150^3 grids (the synthetic composite of the paper's tension-compression
// test), in registers with LDS between the passes.
//
// 150 = 15 x 10: with n = 10 n1 + n2 and k = k1 + 15 k2, a radix-15 pass over
// n1 (lane n2 of a column's ten), the twiddle exp(-2 pi i n2 k1 / 150), and a
// radix-10 pass over n2 (lane k1 of fifteen). The radix-15 and radix-10
// transforms split again as 3 x 5 and 2 x 5 (n = 5 n1' + n2',
// k = k1' + {3, 2} k2'); the length-5 and length-3 transforms are the
// textbook ones on the real and imaginary parts of the roots of unity.
// Twiddles come from one table exp(-2 pi i m / 150), m = 0 .. 149, in LDS.
#pragma once
#include "slab_fft.hpp"

namespace automat {
namespace z150 {

using slab::cd;
constexpr int N = 150;

constexpr double kC5a = 0.30901699437494742410;   // cos(2 pi / 5)
constexpr double kC5b = -0.80901699437494742410;  // cos(4 pi / 5)
constexpr double kS5a = 0.95105651629515357212;   // sin(2 pi / 5)
constexpr double kS5b = 0.58778525229247312917;   // sin(4 pi / 5)
constexpr double kS3 = 0.86602540378443864676;    // sin(2 pi / 3)

__device__ __forceinline__ cd scale(cd a, double s) { return {a.re * s, a.im * s}; }

// X[k] = sum_n x[n] exp(-+2 pi i n k / 5), in place
template <bool INV>
__device__ __forceinline__ void dft5(cd &x0, cd &x1, cd &x2, cd &x3, cd &x4) {
    const cd t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4, t4 = x2 - x3;
    const cd a1 = x0 + scale(t1, kC5a) + scale(t2, kC5b);
    const cd a2 = x0 + scale(t1, kC5b) + scale(t2, kC5a);
    const cd b1 = slab::rot4<INV>(scale(t3, kS5a) + scale(t4, kS5b));
    const cd b2 = slab::rot4<INV>(scale(t3, kS5b) - scale(t4, kS5a));
    x0 = x0 + t1 + t2;
    x1 = a1 + b1;
    x4 = a1 - b1;
    x2 = a2 + b2;
    x3 = a2 - b2;
}

template <bool INV>
__device__ __forceinline__ void dft3(cd &x0, cd &x1, cd &x2) {
    const cd t = x1 + x2;
    const cd a = x0 - scale(t, 0.5);
    const cd b = slab::rot4<INV>(scale(x1 - x2, kS3));
    x0 = x0 + t;
    x1 = a + b;
    x2 = a - b;
}

// length 15 in natural order (3 x 5)
template <bool INV>
__device__ __forceinline__ void dft15(cd *v, const cd *tw) {
    cd y[5][3];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) {
        y[n2][0] = v[n2];
        y[n2][1] = v[5 + n2];
        y[n2][2] = v[10 + n2];
        dft3<INV>(y[n2][0], y[n2][1], y[n2][2]);
#pragma unroll
        for (int k1 = 1; k1 < 3; ++k1) {
            const cd w = tw[10 * n2 * k1];  // exp(-2 pi i n2 k1 / 15)
            y[n2][k1] = slab::twid<INV>(y[n2][k1], w.re, w.im);
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        cd a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1], a4 = y[4][k1];
        dft5<INV>(a0, a1, a2, a3, a4);
        v[k1] = a0;
        v[k1 + 3] = a1;
        v[k1 + 6] = a2;
        v[k1 + 9] = a3;
        v[k1 + 12] = a4;
    }
}

// length 10 in natural order (2 x 5)
template <bool INV>
__device__ __forceinline__ void dft10(cd *v, const cd *tw) {
    cd y[5][2];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) {
        const cd a = v[n2], b = v[5 + n2];
        y[n2][0] = a + b;
        const cd w = tw[15 * n2];  // exp(-2 pi i n2 / 10)
        y[n2][1] = slab::twid<INV>(a - b, w.re, w.im);
    }
#pragma unroll
    for (int k1 = 0; k1 < 2; ++k1) {
        cd a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1], a4 = y[4][k1];
        dft5<INV>(a0, a1, a2, a3, a4);
        v[k1] = a0;
        v[k1 + 2] = a1;
        v[k1 + 4] = a2;
        v[k1 + 6] = a3;
        v[k1 + 8] = a4;
    }
}

// twiddle table exp(-2 pi i m / 150), m = 0 .. 149
__device__ __forceinline__ void init_twiddles(cd *tw) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s, c;
        sincospi((double)m / 75.0, &s, &c);
        tw[m] = {c, -s};
    }
}

// the radix-15 pass of lane n2 (< 10): v[n1] = x[10 n1 + n2] in, twiddled
// partial transforms [k1] out
template <bool INV>
__device__ __forceinline__ void pass15(cd *v, int n2, const cd *tw) {
    dft15<INV>(v, tw);
#pragma unroll
    for (int k1 = 1; k1 < 15; ++k1) {
        const cd w = tw[n2 * k1];
        v[k1] = slab::twid<INV>(v[k1], w.re, w.im);
    }
}

}  // namespace z150
}  // namespace automat
