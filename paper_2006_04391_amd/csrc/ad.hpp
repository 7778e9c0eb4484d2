// ad.hpp -- expression-level automatic differentiation for device code.
//
// The AD design of the paper's Section "Automatic Differentiation on GPUs",
// rebuilt for HIP on gfx950:
//  * operator overloading builds an expression-template tree whose nodes
//    store their arguments (leaves by reference, inner nodes by value); no
//    arithmetic happens until the tree is evaluated (Figure reverse_mode);
//  * every node offers v() (forward evaluation) and back() (reverse
//    propagation of an adjoint); the curiously recurring template pattern
//    resolves the interface at compile time;
//  * there is no tape: back() re-evaluates the argument values and tangents
//    it needs (recomputation instead of taping). Everything is inlined into
//    one kernel, so the compiler sees the whole graph and keeps all AD state
//    in registers;
//  * the second-order extension is written out explicitly for every
//    elementary operation (not by nesting first-order types): back() carries
//    an adjoint bv together with its tangents bt, which gives
//    forward-over-reverse Hessian-vector products ("adjoints of tangents");
//  * the tangents are a vector (forward vector mode): one reverse sweep
//    carries all directions at once, so a full 6x6 Hessian costs one sweep
//    instead of six;
//  * every component of a tangent vector has its own static type, a double
//    or the empty type Zero, and arithmetic on Zero folds away at compile
//    time. Unit seeds therefore cost only the structurally non-zero work, and
//    a first-order sweep (empty tangent vector) is exactly a reverse sweep;
//  * leaves carry a compile-time id. An accumulator picks the ids it
//    collects; adjoints flowing into other leaves are dead code and are
//    removed, which is how partials with respect to one argument group are
//    taken without propagating into the other (mixed-order evaluation).
//
// One deviation from pure recomputation: nodes whose partials need
// transcendental functions or divisions (pow, sqrt, exp, log, division)
// compute them once per sweep in a forward prep() pass and keep them in the
// node. The compiler cannot merge repeated inlined exp/log sequences, so
// recomputing them would repeat the most expensive instructions of the
// sweep; cheap arithmetic is still recomputed.
//
// All functions are __host__ __device__ so the layer can run on the CPU too.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#define AD_FN __host__ __device__ __forceinline__

#include "fastmath.hpp"

// Derivative propagation may be reassociated: a chain of partials that
// scales all six tangent components is then multiplied once instead of per
// component. Only rounding changes (each derivative is a short sum of
// products); primal values keep their written order because they are also
// computed in the files that evaluate the potentials.
#pragma clang fp reassociate(on)

namespace automat {
namespace ad {

// --------------------------------------------------------------------------
// structural zero
// --------------------------------------------------------------------------
struct Zero {};

AD_FN Zero operator+(Zero, Zero) { return {}; }
AD_FN double operator+(Zero, double b) { return b; }
AD_FN double operator+(double a, Zero) { return a; }
AD_FN Zero operator-(Zero, Zero) { return {}; }
AD_FN double operator-(Zero, double b) { return -b; }
AD_FN double operator-(double a, Zero) { return a; }
AD_FN Zero operator-(Zero) { return {}; }
AD_FN Zero operator*(Zero, Zero) { return {}; }
AD_FN Zero operator*(Zero, double) { return {}; }
AD_FN Zero operator*(double, Zero) { return {}; }
AD_FN double &operator+=(double &a, Zero) { return a; }

template <class T>
inline constexpr bool is_zero_v = std::is_same_v<std::decay_t<T>, Zero>;

AD_FN double keep_if(bool c, double x) { return c ? x : 0.0; }
AD_FN Zero keep_if(bool, Zero) { return {}; }

// plain-double square, so potentials can square constant parameters
AD_FN double sq(double x) { return x * x; }

// --------------------------------------------------------------------------
// tangent vectors with per-component static types
// --------------------------------------------------------------------------
template <class... Ts>
struct TV;
template <>
struct TV<> {
    static constexpr int size = 0;
};
template <class T, class... Ts>
struct TV<T, Ts...> {
    static constexpr int size = 1 + sizeof...(Ts);
    T h;
    TV<Ts...> t;
};

template <class H, class... Ts>
AD_FN TV<H, Ts...> cons(H h, const TV<Ts...> &t) {
    return TV<H, Ts...>{h, t};
}

AD_FN TV<> operator+(const TV<> &, const TV<> &) { return {}; }
template <class A, class... As, class B, class... Bs>
AD_FN auto operator+(const TV<A, As...> &a, const TV<B, Bs...> &b) {
    return cons(a.h + b.h, a.t + b.t);
}
AD_FN TV<> operator-(const TV<> &, const TV<> &) { return {}; }
template <class A, class... As, class B, class... Bs>
AD_FN auto operator-(const TV<A, As...> &a, const TV<B, Bs...> &b) {
    return cons(a.h - b.h, a.t - b.t);
}
AD_FN TV<> operator-(const TV<> &) { return {}; }
template <class A, class... As>
AD_FN auto operator-(const TV<A, As...> &a) {
    return cons(-a.h, -a.t);
}
AD_FN TV<> operator*(double, const TV<> &) { return {}; }
template <class A, class... As>
AD_FN auto operator*(double s, const TV<A, As...> &a) {
    return cons(s * a.h, s * a.t);
}
template <class... As>
AD_FN auto operator*(const TV<As...> &a, double s) {
    return s * a;
}
AD_FN TV<> keep_if(bool, const TV<> &) { return {}; }
template <class A, class... As>
AD_FN auto keep_if(bool c, const TV<A, As...> &a) {
    return cons(keep_if(c, a.h), keep_if(c, a.t));
}

// Vector of N structural zeros.
template <int N>
struct zeros_t {
    using type = decltype(cons(Zero{}, typename zeros_t<N - 1>::type{}));
};
template <>
struct zeros_t<0> {
    using type = TV<>;
};
template <int N>
using Zeros = typename zeros_t<N>::type;

// Component J of a tangent vector.
template <int J, class... Ts>
AD_FN auto get(const TV<Ts...> &v) {
    if constexpr (J == 0)
        return v.h;
    else
        return get<J - 1>(v.t);
}

// Unit vector e_K of length N (1.0 at K, Zero elsewhere).
template <int N, int K, int J = 0>
AD_FN auto unit_tv() {
    if constexpr (J == N)
        return TV<>{};
    else if constexpr (J == K)
        return cons(1.0, unit_tv<N, K, J + 1>());
    else
        return cons(Zero{}, unit_tv<N, K, J + 1>());
}

// --------------------------------------------------------------------------
// directions (tangent seeds of the leaves)
// --------------------------------------------------------------------------

// No direction: first-order reverse sweep (empty tangent vectors).
struct NoDir {
    static constexpr int width = 0;
    template <int ID>
    AD_FN TV<> seed() const { return {}; }
};

// The N unit directions of leaves BASE .. BASE+N-1, all at once.
template <int N, int BASE = 0>
struct UnitDirs {
    static constexpr int width = N;
    template <int ID>
    AD_FN auto seed() const {
        if constexpr (ID >= BASE && ID < BASE + N)
            return unit_tv<N, ID - BASE>();
        else
            return Zeros<N>{};
    }
};

// One runtime direction d on leaves BASE .. BASE+N-1.
template <int N, int BASE = 0>
struct VecDir {
    static constexpr int width = 1;
    double d[N];
    template <int ID>
    AD_FN auto seed() const {
        if constexpr (ID >= BASE && ID < BASE + N)
            return TV<double>{d[ID - BASE], TV<>{}};
        else
            return Zeros<1>{};
    }
};

// --------------------------------------------------------------------------
// accumulators (where leaf adjoints go)
// --------------------------------------------------------------------------

// First-order adjoints of leaves BASE .. BASE+N-1.
template <int N, int BASE = 0>
struct Grad {
    double g[N];
    AD_FN Grad() {
        for (int i = 0; i < N; ++i) g[i] = 0.0;
    }
    template <int ID, class B, class BT>
    AD_FN void acc(B bv, const BT &) {
        if constexpr (ID >= BASE && ID < BASE + N) g[ID - BASE] += bv;
    }
};

// Adjoint tangents of leaves BASE .. BASE+N-1 for a one-direction sweep
// (a Hessian-vector product), optionally with the first-order adjoints.
template <int N, int BASE = 0>
struct GradT {
    double g[N];   // tangent of the adjoint
    double g1[N];  // first-order adjoint
    AD_FN GradT() {
        for (int i = 0; i < N; ++i) g[i] = g1[i] = 0.0;
    }
    template <int ID, class B, class BT>
    AD_FN void acc(B bv, const BT &bt) {
        if constexpr (ID >= BASE && ID < BASE + N) {
            g[ID - BASE] += bt.h;
            g1[ID - BASE] += bv;
        }
    }
};

// Rows of a Hessian block: leaves BASE .. BASE+N-1 times the W directions
// of the sweep, plus the first-order adjoints.
template <int N, int W, int BASE = 0>
struct HessRows {
    double H[N][W];
    double g[N];
    AD_FN HessRows() {
        for (int i = 0; i < N; ++i) {
            g[i] = 0.0;
            for (int j = 0; j < W; ++j) H[i][j] = 0.0;
        }
    }
    template <int I, int J, class... Ts>
    AD_FN void put(const TV<Ts...> &bt) {
        if constexpr (J < W) {
            H[I][J] += get<J>(bt);
            put<I, J + 1>(bt);
        }
    }
    template <int ID, class B, class BT>
    AD_FN void acc(B bv, const BT &bt) {
        if constexpr (ID >= BASE && ID < BASE + N) {
            g[ID - BASE] += bv;
            put<ID - BASE, 0>(bt);
        }
    }
};

// --------------------------------------------------------------------------
// expression interface (CRTP)
// --------------------------------------------------------------------------
template <class D>
struct Expr {
    AD_FN const D &self() const { return static_cast<const D &>(*this); }
};

template <class T>
struct is_expr : std::is_base_of<Expr<T>, T> {};

// Active leaf with compile-time id.
template <int ID>
struct Var : Expr<Var<ID>> {
    double val;
    AD_FN Var() : val(0.0) {}
    AD_FN explicit Var(double x) : val(x) {}
    AD_FN void prep() const {}
    AD_FN double v() const { return val; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return d.template seed<ID>(); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &, B bv, const BT &bt) const {
        adj.template acc<ID>(bv, bt);
    }
};

// Passive constant (stored by value).
struct Cst : Expr<Cst> {
    double val;
    AD_FN explicit Cst(double x) : val(x) {}
    AD_FN void prep() const {}
    AD_FN double v() const { return val; }
    template <class Dir>
    AD_FN auto t(const Dir &) const { return Zeros<Dir::width>{}; }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &, const Dir &, B, const BT &) const {}
};

template <class T>
struct leaf_trait {
    static constexpr bool value = false;
};
template <int ID>
struct leaf_trait<Var<ID>> {
    static constexpr bool value = true;
};

// Leaves are referenced, inner nodes copied.
template <class T>
using Store = std::conditional_t<leaf_trait<T>::value, const T &, const T>;

template <class T>
AD_FN decltype(auto) as_expr(const T &x) {
    if constexpr (std::is_arithmetic_v<T>)
        return Cst(static_cast<double>(x));
    else
        return (x);
}
template <class T>
using expr_t = std::decay_t<decltype(as_expr(std::declval<const T &>()))>;

// --------------------------------------------------------------------------
// binary operations
// --------------------------------------------------------------------------
template <class L, class R>
struct Add : Expr<Add<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Add(const L &a, const R &b) : l(a), r(b) {}
    AD_FN void prep() const {
        l.prep();
        r.prep();
    }
    AD_FN double v() const { return l.v() + r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) + r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        l.back(adj, d, bv, bt);
        r.back(adj, d, bv, bt);
    }
};

template <class L, class R>
struct Sub : Expr<Sub<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Sub(const L &a, const R &b) : l(a), r(b) {}
    AD_FN void prep() const {
        l.prep();
        r.prep();
    }
    AD_FN double v() const { return l.v() - r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) - r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        l.back(adj, d, bv, bt);
        r.back(adj, d, -bv, -bt);
    }
};

// d(lr) = r dl + l dr; the only second derivative is d2/dl dr = 1
template <class L, class R>
struct Mul : Expr<Mul<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Mul(const L &a, const R &b) : l(a), r(b) {}
    AD_FN void prep() const {
        l.prep();
        r.prep();
    }
    AD_FN double v() const { return l.v() * r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) * r.v() + l.v() * r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        const double lv = l.v(), rv = r.v();
        l.back(adj, d, bv * rv, bt * rv + bv * r.t(d));
        r.back(adj, d, bv * lv, bt * lv + bv * l.t(d));
    }
};

// q = l / r: dq = (dl - q dr) / r; partials 1/r and -q/r with tangents
// -dr/r^2 and -(dl - 2 q dr)/r^2. The reciprocal is kept from prep().
template <class L, class R>
struct Div : Expr<Div<L, R>> {
    Store<L> l;
    Store<R> r;
    mutable double ir;
    AD_FN Div(const L &a, const R &b) : l(a), r(b), ir(0.0) {}
    AD_FN void prep() const {
        l.prep();
        r.prep();
        ir = fm::rcp(r.v());
    }
    AD_FN double v() const { return l.v() * ir; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return (l.t(d) - (l.v() * ir) * r.t(d)) * ir; }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        const double q = l.v() * ir;
        auto lt = l.t(d);
        auto rt = r.t(d);
        l.back(adj, d, bv * ir, bt * ir - bv * (rt * (ir * ir)));
        r.back(adj, d, bv * (-q * ir), bt * (-q * ir) - bv * ((lt - (2.0 * q) * rt) * (ir * ir)));
    }
};

// --------------------------------------------------------------------------
// unary operations
// --------------------------------------------------------------------------
template <class A>
struct Neg : Expr<Neg<A>> {
    Store<A> a;
    AD_FN explicit Neg(const A &x) : a(x) {}
    AD_FN void prep() const { a.prep(); }
    AD_FN double v() const { return -a.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return -a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        a.back(adj, d, -bv, -bt);
    }
};

// x^2
template <class A>
struct Square : Expr<Square<A>> {
    Store<A> a;
    AD_FN explicit Square(const A &x) : a(x) {}
    AD_FN void prep() const { a.prep(); }
    AD_FN double v() const {
        const double x = a.v();
        return x * x;
    }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return (2.0 * a.v()) * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        const double x2 = 2.0 * a.v();
        a.back(adj, d, bv * x2, bt * x2 + (2.0 * bv) * a.t(d));
    }
};

// sqrt(x); the derivative is taken as 0 where x = 0, so that a zero
// adjoint arriving at a cone point (e.g. the equivalent stress of a
// hydrostatic state) propagates as zero instead of 0 * inf.
template <class A>
struct Sqrt : Expr<Sqrt<A>> {
    Store<A> a;
    mutable double y, iy;
    AD_FN explicit Sqrt(const A &x) : a(x), y(0.0), iy(0.0) {}
    AD_FN void prep() const {
        a.prep();
        const double x = a.v();
        const double r = x > 0.0 ? fm::rsqrt(x) : 0.0;
        y = x * r;
        iy = r;
    }
    AD_FN double v() const { return y; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return (0.5 * iy) * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        const double c = 0.5 * iy;
        a.back(adj, d, bv * c, bt * c + (bv * (-0.25 * iy * iy * iy)) * a.t(d));
    }
};

// max(x, 0): derivative 1 for x > 0, else 0; second derivative 0
template <class A>
struct Pos : Expr<Pos<A>> {
    Store<A> a;
    AD_FN explicit Pos(const A &x) : a(x) {}
    AD_FN void prep() const { a.prep(); }
    AD_FN double v() const {
        const double x = a.v();
        return x > 0.0 ? x : 0.0;
    }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return keep_if(a.v() > 0.0, a.t(d)); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        const bool on = a.v() > 0.0;
        a.back(adj, d, keep_if(on, bv), keep_if(on, bt));
    }
};

template <class A>
struct Exp : Expr<Exp<A>> {
    Store<A> a;
    mutable double y;
    AD_FN explicit Exp(const A &x) : a(x), y(0.0) {}
    AD_FN void prep() const {
        a.prep();
        y = fm::exp(a.v());
    }
    AD_FN double v() const { return y; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return y * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        a.back(adj, d, bv * y, bt * y + (bv * y) * a.t(d));
    }
};

template <class A>
struct Log : Expr<Log<A>> {
    Store<A> a;
    mutable double y, ix;
    AD_FN explicit Log(const A &x) : a(x), y(0.0), ix(0.0) {}
    AD_FN void prep() const {
        a.prep();
        y = fm::log(a.v());
        ix = fm::rcp(a.v());
    }
    AD_FN double v() const { return y; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return ix * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        a.back(adj, d, bv * ix, bt * ix - (bv * ix * ix) * a.t(d));
    }
};

// u^p for u >= 0 and p >= 1, both differentiable.
// For u > 0: y = exp(p log u), y_u = p y / u, y_p = y log u,
//   y_uu = (p - 1) y_u / u, y_up = y_u log u + y / u, y_pp = y_p log u.
// At u = 0 the one-sided limits for p >= 1 are used: y = 0, y_p = 0,
// y_u = [p == 1], y_uu = 2 [p == 2], y_up = 0, y_pp = 0 (for 1 < p < 2 the
// true y_uu is unbounded; it only ever multiplies a zero tangent there).
template <class U, class P>
struct Pow : Expr<Pow<U, P>> {
    Store<U> u;
    Store<P> p;
    mutable double y, yu, yp, yuu, yup, ypp;
    AD_FN Pow(const U &a, const P &b) : u(a), p(b), y(0), yu(0), yp(0), yuu(0), yup(0), ypp(0) {}
    AD_FN void prep() const {
        u.prep();
        p.prep();
        const double uv = u.v(), pv = p.v();
        // Every branch fills locals and the members are assigned once, so
        // the node stays in registers.
        double Y = 0.0, Yu = 0.0, Yp = 0.0, Yuu = 0.0, Yup = 0.0, Ypp = 0.0;
        if (uv > 0.0) {
            const double lu = fm::log(uv);
            const double iu = fm::rcp(uv);
            Y = fm::exp(pv * lu);
            Yu = pv * Y * iu;
            Yp = Y * lu;
            Yuu = (pv - 1.0) * Yu * iu;
            Yup = Yu * lu + Y * iu;
            Ypp = Yp * lu;
        } else {
            Yu = pv == 1.0 ? 1.0 : 0.0;
            Yuu = pv == 2.0 ? 2.0 : 0.0;
        }
        y = Y;
        yu = Yu;
        yp = Yp;
        yuu = Yuu;
        yup = Yup;
        ypp = Ypp;
    }
    AD_FN double v() const { return y; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return yu * u.t(d) + yp * p.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, const BT &bt) const {
        auto ut = u.t(d);
        auto pt = p.t(d);
        u.back(adj, d, bv * yu, bt * yu + bv * (yuu * ut + yup * pt));
        p.back(adj, d, bv * yp, bt * yp + bv * (yup * ut + ypp * pt));
    }
};

// --------------------------------------------------------------------------
// operator overloads and functions (build nodes, evaluate nothing)
// --------------------------------------------------------------------------
template <class T>
inline constexpr bool ad_operand_v = is_expr<std::decay_t<T>>::value || std::is_arithmetic_v<T>;
template <class L, class R>
inline constexpr bool ad_binary_v =
    ad_operand_v<L> && ad_operand_v<R> &&
    (is_expr<std::decay_t<L>>::value || is_expr<std::decay_t<R>>::value);

#define AD_BINARY(OP, NODE)                                                          \
    template <class L, class R, std::enable_if_t<ad_binary_v<L, R>, int> = 0>        \
    AD_FN auto OP(const L &a, const R &b) {                                          \
        return NODE<expr_t<L>, expr_t<R>>(as_expr(a), as_expr(b));                   \
    }
AD_BINARY(operator+, Add)
AD_BINARY(operator-, Sub)
AD_BINARY(operator*, Mul)
AD_BINARY(operator/, Div)
AD_BINARY(pow, Pow)
#undef AD_BINARY

#define AD_UNARY(FN, NODE)                                                           \
    template <class A, std::enable_if_t<is_expr<A>::value, int> = 0>                 \
    AD_FN auto FN(const A &a) {                                                      \
        return NODE<A>(a);                                                           \
    }
AD_UNARY(operator-, Neg)
AD_UNARY(sq, Square)
AD_UNARY(sqrt, Sqrt)
AD_UNARY(pos, Pos)
AD_UNARY(exp, Exp)
AD_UNARY(log, Log)
#undef AD_UNARY

// --------------------------------------------------------------------------
// drivers
// --------------------------------------------------------------------------

// Value only.
template <class E>
AD_FN double value(const E &e) {
    e.prep();
    return e.v();
}

// Value and first-order adjoints (seed 1 at the root).
template <class E, class Adj>
AD_FN double value_grad(const E &e, Adj &adj) {
    e.prep();
    e.back(adj, NoDir{}, 1.0, TV<>{});
    return e.v();
}

// Forward-over-reverse sweep in the directions of d: the accumulator
// receives first-order adjoints and their tangents (Hessian times the
// direction vectors). Returns the value.
template <class E, class Dir, class Adj>
AD_FN double sweep2(const E &e, const Dir &d, Adj &adj) {
    e.prep();
    e.back(adj, d, 1.0, Zeros<Dir::width>{});
    return e.v();
}

// Value, gradient and packed lower-triangular Hessian (entry (i, j), j <= i,
// at i (i + 1) / 2 + j) over the six leaves BASE .. BASE+5, in one sweep.
template <int BASE, class E>
AD_FN double value_grad_hess6(const E &e, double *g, double *Hp) {
    HessRows<6, 6, BASE> acc;
    const double val = sweep2(e, UnitDirs<6, BASE>{}, acc);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        g[i] = acc.g[i];
#pragma unroll
        for (int j = 0; j <= i; ++j) Hp[i * (i + 1) / 2 + j] = acc.H[i][j];
    }
    return val;
}

// Full block d2 e / (d x_{ROW+i} d x_{COL+j}) in one sweep.
template <int ROW, int COL, class E>
AD_FN void hessian_block6(const E &e, double (&H)[6][6]) {
    HessRows<6, 6, ROW> acc;
    sweep2(e, UnitDirs<6, COL>{}, acc);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) H[i][j] = acc.H[i][j];
}

}  // namespace ad
}  // namespace automat

#pragma clang fp reassociate(off)
