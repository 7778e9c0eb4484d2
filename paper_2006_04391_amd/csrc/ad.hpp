// ad.hpp -- expression-level automatic differentiation for device code.
//
// The AD design of the paper's Section "Automatic Differentiation on GPUs",
// rebuilt for HIP:
//  * operator overloading builds an expression-template tree whose nodes
//    store their arguments (leaves by reference, inner nodes by value); no
//    arithmetic happens until the tree is evaluated (Figure reverse_mode);
//  * every node offers v() (forward evaluation) and back() (reverse
//    propagation of an adjoint); the curiously recurring template pattern
//    resolves the interface at compile time;
//  * there is no tape: back() re-evaluates the argument subtrees it needs
//    (recomputation instead of taping). Everything is inlined into one
//    kernel, so the compiler sees the whole graph, merges the repeated
//    subexpressions and keeps all AD state in registers;
//  * the second-order extension is written out explicitly for every
//    elementary operation (not by nesting first-order types): back() carries
//    an adjoint bv together with its tangent bt in one direction, which
//    gives forward-over-reverse Hessian-vector products ("adjoints of
//    tangents");
//  * a direction object supplies each leaf's tangent seed. Seeds that are
//    zero by construction have the empty type Zero, and arithmetic on Zero
//    folds away at compile time, so a unit-direction Hessian pass costs only
//    the non-zero work and a first-order pass (all seeds Zero) costs exactly a
//    reverse sweep;
//  * leaves carry a compile-time id. An accumulator picks the ids it
//    collects; adjoints flowing into other leaves are dead code and are
//    removed, which is how partials with respect to one argument group are
//    taken without propagating into the other (mixed-order evaluation).
//
// All functions are __host__ __device__ so the layer can be exercised on
// the CPU as well.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#define AD_FN __host__ __device__ __forceinline__

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
AD_FN Zero operator/(Zero, double) { return {}; }
AD_FN double &operator+=(double &a, Zero) { return a; }

template <class T>
inline constexpr bool is_zero_v = std::is_same_v<std::decay_t<T>, Zero>;

// c ? x : 0 for a double, Zero stays Zero
AD_FN double keep_if(bool c, double x) { return c ? x : 0.0; }
AD_FN Zero keep_if(bool, Zero) { return {}; }

// plain-double square, so potentials can square constant parameters
AD_FN double sq(double x) { return x * x; }

// --------------------------------------------------------------------------
// directions (tangent seeds of the leaves)
// --------------------------------------------------------------------------

// No direction: first-order reverse sweep.
struct NoDir {
    template <int ID>
    AD_FN Zero seed() const { return {}; }
};

// Unit direction e_{BASE+K}: seed 1 on leaf BASE+K, Zero elsewhere.
template <int K, int BASE = 0>
struct UnitDir {
    template <int ID>
    AD_FN auto seed() const {
        if constexpr (ID == BASE + K)
            return 1.0;
        else
            return Zero{};
    }
};

// Runtime direction on leaves BASE .. BASE+N-1, Zero elsewhere.
template <int N, int BASE = 0>
struct VecDir {
    double d[N];
    template <int ID>
    AD_FN auto seed() const {
        if constexpr (ID >= BASE && ID < BASE + N)
            return d[ID - BASE];
        else
            return Zero{};
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
    AD_FN void acc(B bv, BT) {
        if constexpr (ID >= BASE && ID < BASE + N) g[ID - BASE] += bv;
    }
};

// Tangents of the adjoints (Hessian-vector products) of leaves
// BASE .. BASE+N-1.
template <int N, int BASE = 0>
struct GradT {
    double g[N];
    AD_FN GradT() {
        for (int i = 0; i < N; ++i) g[i] = 0.0;
    }
    template <int ID, class B, class BT>
    AD_FN void acc(B, BT bt) {
        if constexpr (ID >= BASE && ID < BASE + N) g[ID - BASE] += bt;
    }
};

// Both at once.
template <int N, int BASE = 0>
struct Grad2 {
    double g[N], h[N];
    AD_FN Grad2() {
        for (int i = 0; i < N; ++i) g[i] = h[i] = 0.0;
    }
    template <int ID, class B, class BT>
    AD_FN void acc(B bv, BT bt) {
        if constexpr (ID >= BASE && ID < BASE + N) {
            g[ID - BASE] += bv;
            h[ID - BASE] += bt;
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
    static constexpr bool is_leaf = true;
    double val;
    AD_FN Var() : val(0.0) {}
    AD_FN explicit Var(double x) : val(x) {}
    AD_FN double v() const { return val; }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return d.template seed<ID>(); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &, B bv, BT bt) const {
        adj.template acc<ID>(bv, bt);
    }
};

// Passive constant (stored by value).
struct Cst : Expr<Cst> {
    static constexpr bool is_leaf = false;
    double val;
    AD_FN explicit Cst(double x) : val(x) {}
    AD_FN double v() const { return val; }
    template <class Dir>
    AD_FN Zero t(const Dir &) const { return {}; }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &, const Dir &, B, BT) const {}
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

// wrap a double operand into a constant node
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
    AD_FN double v() const { return l.v() + r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) + r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        l.back(adj, d, bv, bt);
        r.back(adj, d, bv, bt);
    }
};

template <class L, class R>
struct Sub : Expr<Sub<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Sub(const L &a, const R &b) : l(a), r(b) {}
    AD_FN double v() const { return l.v() - r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) - r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        l.back(adj, d, bv, bt);
        r.back(adj, d, -bv, -bt);
    }
};

// d(lr) = r dl + l dr; second order: d2/dl dr = 1
template <class L, class R>
struct Mul : Expr<Mul<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Mul(const L &a, const R &b) : l(a), r(b) {}
    AD_FN double v() const { return l.v() * r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return l.t(d) * r.v() + l.v() * r.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double lv = l.v(), rv = r.v();
        l.back(adj, d, bv * rv, bt * rv + bv * r.t(d));
        r.back(adj, d, bv * lv, bt * lv + bv * l.t(d));
    }
};

// d(l/r) = dl / r - l dr / r^2
template <class L, class R>
struct Div : Expr<Div<L, R>> {
    Store<L> l;
    Store<R> r;
    AD_FN Div(const L &a, const R &b) : l(a), r(b) {}
    AD_FN double v() const { return l.v() / r.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const {
        const double ir = 1.0 / r.v();
        return (l.t(d) - (l.v() * ir) * r.t(d)) * ir;
    }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double ir = 1.0 / r.v();
        const double q = l.v() * ir;               // the quotient
        auto lt = l.t(d);
        auto rt = r.t(d);
        auto qt = (lt - q * rt) * ir;              // tangent of the quotient
        // d/dl = 1/r, d/dr = -q/r; their tangents -rt/r^2 and -(qt r - q rt)/r^2
        l.back(adj, d, bv * ir, bt * ir - bv * (rt * (ir * ir)));
        r.back(adj, d, bv * (-q * ir), bt * (-q * ir) - bv * ((qt - q * ir * rt) * ir));
    }
};

// --------------------------------------------------------------------------
// unary operations
// --------------------------------------------------------------------------
template <class A>
struct Neg : Expr<Neg<A>> {
    Store<A> a;
    AD_FN explicit Neg(const A &x) : a(x) {}
    AD_FN double v() const { return -a.v(); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return -a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        a.back(adj, d, -bv, -bt);
    }
};

// x^2
template <class A>
struct Square : Expr<Square<A>> {
    Store<A> a;
    AD_FN explicit Square(const A &x) : a(x) {}
    AD_FN double v() const {
        const double x = a.v();
        return x * x;
    }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return (2.0 * a.v()) * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double x = a.v();
        a.back(adj, d, bv * (2.0 * x), bt * (2.0 * x) + (2.0 * bv) * a.t(d));
    }
};

// sqrt(x); the derivative is taken as 0 where x = 0, so that a zero
// adjoint arriving at a cone point (e.g. the equivalent stress of a
// hydrostatic state) propagates as zero instead of 0 * inf.
template <class A>
struct Sqrt : Expr<Sqrt<A>> {
    Store<A> a;
    AD_FN explicit Sqrt(const A &x) : a(x) {}
    AD_FN double v() const { return ::sqrt(a.v()); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const {
        const double y = ::sqrt(a.v());
        const double c = y > 0.0 ? 0.5 / y : 0.0;
        return c * a.t(d);
    }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double y = ::sqrt(a.v());
        const double iy = y > 0.0 ? 1.0 / y : 0.0;
        const double c = 0.5 * iy;                 // dy/dx
        auto ct = (-0.25 * iy * iy * iy) * a.t(d); // tangent of dy/dx
        a.back(adj, d, bv * c, bt * c + bv * ct);
    }
};

// max(x, 0): derivative 1 for x > 0, else 0; second derivative 0
template <class A>
struct Pos : Expr<Pos<A>> {
    Store<A> a;
    AD_FN explicit Pos(const A &x) : a(x) {}
    AD_FN double v() const {
        const double x = a.v();
        return x > 0.0 ? x : 0.0;
    }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return keep_if(a.v() > 0.0, a.t(d)); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const bool on = a.v() > 0.0;
        a.back(adj, d, keep_if(on, bv), keep_if(on, bt));
    }
};

template <class A>
struct Exp : Expr<Exp<A>> {
    Store<A> a;
    AD_FN explicit Exp(const A &x) : a(x) {}
    AD_FN double v() const { return ::exp(a.v()); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return ::exp(a.v()) * a.t(d); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double y = ::exp(a.v());
        a.back(adj, d, bv * y, bt * y + (bv * y) * a.t(d));
    }
};

template <class A>
struct Log : Expr<Log<A>> {
    Store<A> a;
    AD_FN explicit Log(const A &x) : a(x) {}
    AD_FN double v() const { return ::log(a.v()); }
    template <class Dir>
    AD_FN auto t(const Dir &d) const { return a.t(d) / a.v(); }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const double ix = 1.0 / a.v();
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
    AD_FN Pow(const U &a, const P &b) : u(a), p(b) {}

    struct Partials {
        double y, yu, yp, yuu, yup, ypp;
    };
    AD_FN static Partials partials(double uv, double pv) {
        Partials r;
        if (uv > 0.0) {
            const double lu = ::log(uv);
            const double iu = 1.0 / uv;
            r.y = ::exp(pv * lu);
            r.yu = pv * r.y * iu;
            r.yp = r.y * lu;
            r.yuu = (pv - 1.0) * r.yu * iu;
            r.yup = r.yu * lu + r.y * iu;
            r.ypp = r.yp * lu;
        } else {
            r.y = 0.0;
            r.yp = 0.0;
            r.yu = pv == 1.0 ? 1.0 : 0.0;
            r.yuu = pv == 2.0 ? 2.0 : 0.0;
            r.yup = 0.0;
            r.ypp = 0.0;
        }
        return r;
    }
    AD_FN double v() const {
        const double uv = u.v();
        return uv > 0.0 ? ::exp(p.v() * ::log(uv)) : 0.0;
    }
    template <class Dir>
    AD_FN auto t(const Dir &d) const {
        const Partials r = partials(u.v(), p.v());
        return r.yu * u.t(d) + r.yp * p.t(d);
    }
    template <class Adj, class Dir, class B, class BT>
    AD_FN void back(Adj &adj, const Dir &d, B bv, BT bt) const {
        const Partials r = partials(u.v(), p.v());
        auto ut = u.t(d);
        auto pt = p.t(d);
        u.back(adj, d, bv * r.yu, bt * r.yu + bv * (r.yuu * ut + r.yup * pt));
        p.back(adj, d, bv * r.yp, bt * r.yp + bv * (r.yup * ut + r.ypp * pt));
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

// Value and first-order adjoints (seed 1 at the root).
template <class E, class Adj>
AD_FN double value_grad(const E &e, Adj &adj) {
    e.back(adj, NoDir{}, 1.0, Zero{});
    return e.v();
}

// Adjoint tangents in direction d: accumulates (Hessian . d) into adj.
template <class E, class Dir, class Adj>
AD_FN void hess_vec(const E &e, const Dir &d, Adj &adj) {
    e.back(adj, d, 1.0, Zero{});
}

// Directional derivative (forward tangent) of the value.
template <class E, class Dir>
AD_FN double tangent(const E &e, const Dir &d) {
    auto t = e.t(d);
    if constexpr (is_zero_v<decltype(t)>)
        return 0.0;
    else
        return t;
}

// Hessian block d2 e / (d x_{ROW+i} d x_{COL+j}), i, j < N, by N unit
// passes. Column j of the block is one Hessian-vector product.
template <int N, int ROW, int COL, class E, int J = 0>
AD_FN void hessian_block(const E &e, double (&H)[N][N]) {
    if constexpr (J < N) {
        GradT<N, ROW> acc;
        hess_vec(e, UnitDir<J, COL>{}, acc);
        for (int i = 0; i < N; ++i) H[i][J] = acc.g[i];
        hessian_block<N, ROW, COL, E, J + 1>(e, H);
    }
}

// Lower triangle (packed row-major: (i, j), j <= i at i (i + 1) / 2 + j) of
// a symmetric Hessian block over leaves BASE .. BASE+5.
template <int BASE, class E, int J = 0>
AD_FN void hessian_sym6(const E &e, double (&Hp)[21]) {
    if constexpr (J < 6) {
        GradT<6, BASE> acc;
        hess_vec(e, UnitDir<J, BASE>{}, acc);
#pragma unroll
        for (int i = J; i < 6; ++i) Hp[i * (i + 1) / 2 + J] = acc.g[i];
        hessian_sym6<BASE, E, J + 1>(e, Hp);
    }
}

}  // namespace ad
}  // namespace automat
