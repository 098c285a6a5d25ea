// Register-resident small FFTs for the collision kernels (host + device).
//
// A length-N transform lives in an array of N complex values; every index is a
// compile-time constant after template expansion, so the arrays map to
// registers and all permutations are free.  The recursion is a mixed-radix
// (4, 2, 3) decimation in time; twiddle factors are exact compile-time
// constants computed in double precision (then rounded to the working type),
// and multiplications by 1, -1 and +-i are removed at compile time.  In the
// radix-4 combinations each nontrivial twiddle is factored as g (1 + i t) or
// g (t + i) (Linzer-Feig), so that g folds into the butterfly's additions as
// FMAs: 24 instead of 28 instructions per twiddled radix-4 butterfly.
//
//   fft<T, N, SIGN>(x):  x[k] <- sum_n x[n] exp(SIGN * 2 pi i n k / N)   (unnormalised)
#pragma once

#include <cstdint>
#include <type_traits>
#include <utility>

#if defined(__HIPCC__)
#define FKS_HD __host__ __device__ __forceinline__
#else
#define FKS_HD inline
#endif

namespace fks {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
FKS_HD cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
FKS_HD cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
// a * (s i), s = +-1
template <typename T, int S>
FKS_HD cx<T> cmul_i(cx<T> a) {
    if constexpr (S > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}

// ---------------------------------------------------------------------------
// compile-time trigonometry (double): sin/cos(2 pi num/den) by exact octant
// reduction and Taylor series on [0, pi/4] (within a few ulp of double)
// ---------------------------------------------------------------------------
namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double sin_red(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k <= 12; ++k) {
        term *= -x2 / double((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}
constexpr double cos_red(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k <= 12; ++k) {
        term *= -x2 / double((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}
// sin and cos of 2 pi num / den
struct sc { double s, c; };
constexpr sc sincos2pi(long num, long den) {
    num %= den;
    if (num < 0) num += den;
    // angle = (pi/4) * (8 num / den): octant o, fraction r/den of an octant
    long e8 = 8 * num;
    long o = e8 / den;
    long r = e8 - o * den;              // in [0, den)
    double a = (kPi / 4.0) * double(r) / double(den);           // in [0, pi/4)
    double b = (kPi / 4.0) * double(den - r) / double(den);     // pi/4 - a, exact complement
    double s = 0, c = 0;
    switch (o) {
        case 0: s = sin_red(a);  c = cos_red(a);  break;
        case 1: s = cos_red(b);  c = sin_red(b);  break;
        case 2: s = cos_red(a);  c = -sin_red(a); break;
        case 3: s = sin_red(b);  c = -cos_red(b); break;
        case 4: s = -sin_red(a); c = -cos_red(a); break;
        case 5: s = -cos_red(b); c = -sin_red(b); break;
        case 6: s = -cos_red(a); c = sin_red(a);  break;
        default: s = -sin_red(b); c = cos_red(b); break;
    }
    return {s, c};
}
}  // namespace ct

// compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1
template <typename F, int... Is>
FKS_HD void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
FKS_HD void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// multiply by W = exp(SIGN * 2 pi i E / N)
template <typename T, int SIGN, int N, int E>
FKS_HD cx<T> twiddle(cx<T> a) {
    constexpr int e = ((E % N) + N) % N;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (2 * e == N) {
        return {-a.x, -a.y};
    } else if constexpr (4 * e == N) {
        return cmul_i<T, SIGN>(a);
    } else if constexpr (4 * e == 3 * N) {
        return cmul_i<T, -SIGN>(a);
    } else {
        constexpr ct::sc w = ct::sincos2pi(e, N);
        constexpr T c = T(w.c);
        constexpr T s = T(SIGN > 0 ? w.s : -w.s);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// Twiddle factored as W = g (1 + i t) or g (t + i) with |t| <= 1 and the larger of
// |cos|, |sin| as g (Linzer-Feig): W a = g v with v = pre(a) costing two FMAs,
// and the radix-4 butterfly absorbs g into its additions as FMAs.
template <typename T, int SIGN, int N, int E>
struct ScaledTwiddle {
    static constexpr int e = ((E % N) + N) % N;
    static constexpr bool trivial = e == 0 || 2 * e == N || 4 * e == N || 4 * e == 3 * N;
    static constexpr ct::sc w = ct::sincos2pi(e, N);
    static constexpr double c = w.c;
    static constexpr double s = SIGN > 0 ? w.s : -w.s;
    static constexpr bool cos_major = (c < 0 ? -c : c) >= (s < 0 ? -s : s);
    static constexpr T g = trivial ? T(1) : T(cos_major ? c : s);
    static constexpr T t = trivial ? T(0) : T(cos_major ? s / c : c / s);
    FKS_HD static cx<T> pre(cx<T> a) {
        if constexpr (trivial) {
            return twiddle<T, SIGN, N, E>(a);
        } else if constexpr (cos_major) {   // W a = c ((x - t y) + i (y + t x))
            return {a.x - t * a.y, a.y + t * a.x};
        } else {                            // W a = s ((t x - y) + i (x + t y))
            return {t * a.x - a.y, a.x + t * a.y};
        }
    }
};

template <int N>
constexpr int first_radix() {
    return (N % 4 == 0) ? 4 : (N % 2 == 0 ? 2 : (N % 3 == 0 ? 3 : N));
}

// radix-R butterfly in place: u[q] <- sum_r u[r] exp(SIGN 2 pi i r q / R)
template <typename T, int R, int SIGN>
FKS_HD void butterfly(cx<T>* u) {
    if constexpr (R == 2) {
        cx<T> a = u[0], b = u[1];
        u[0] = cadd(a, b);
        u[1] = csub(a, b);
    } else if constexpr (R == 4) {
        cx<T> a = cadd(u[0], u[2]);
        cx<T> b = csub(u[0], u[2]);
        cx<T> c = cadd(u[1], u[3]);
        cx<T> d = cmul_i<T, SIGN>(csub(u[1], u[3]));
        u[0] = cadd(a, c);
        u[2] = csub(a, c);
        u[1] = cadd(b, d);
        u[3] = csub(b, d);
    } else if constexpr (R == 3) {
        constexpr T h = T(0.8660254037844386467637231707529362);  // sqrt(3)/2
        cx<T> s = cadd(u[1], u[2]);
        cx<T> d = csub(u[1], u[2]);
        cx<T> m = {u[0].x - T(0.5) * s.x, u[0].y - T(0.5) * s.y};
        cx<T> t = cmul_i<T, SIGN>(cx<T>{h * d.x, h * d.y});
        u[0] = cadd(u[0], s);
        u[1] = cadd(m, t);
        u[2] = csub(m, t);
    } else {
        static_assert(R == 2 || R == 3 || R == 4, "unsupported radix");
    }
}

// one output group k of a radix-R combination: y[k + M q], q < R, from sub[r][k]
template <typename T, int N, int SIGN, int R, int M, int k>
FKS_HD void combine(const cx<T> (&sub)[R][M], cx<T>* y) {
    if constexpr (R == 4 && !(ScaledTwiddle<T, SIGN, N, k>::trivial &&
                              ScaledTwiddle<T, SIGN, N, 2 * k>::trivial &&
                              ScaledTwiddle<T, SIGN, N, 3 * k>::trivial)) {
        using W1 = ScaledTwiddle<T, SIGN, N, k>;
        using W2 = ScaledTwiddle<T, SIGN, N, 2 * k>;
        using W3 = ScaledTwiddle<T, SIGN, N, 3 * k>;
        const cx<T> u0 = sub[0][k];
        const cx<T> v1 = W1::pre(sub[1][k]), v2 = W2::pre(sub[2][k]), v3 = W3::pre(sub[3][k]);
        constexpr T g1 = W1::g, g2 = W2::g, g3 = W3::g;
        const cx<T> a = {u0.x + g2 * v2.x, u0.y + g2 * v2.y};
        const cx<T> b = {u0.x - g2 * v2.x, u0.y - g2 * v2.y};
        cx<T> c, d;
        if constexpr (g1 == g3) {         // c = g (v1 + v3), d = g (v1 - v3)
            const cx<T> sp = cadd(v1, v3), sm = csub(v1, v3);
            const cx<T> dm = cmul_i<T, SIGN>(sm);
            y[k] = {a.x + g1 * sp.x, a.y + g1 * sp.y};
            y[k + 2 * M] = {a.x - g1 * sp.x, a.y - g1 * sp.y};
            y[k + M] = {b.x + g1 * dm.x, b.y + g1 * dm.y};
            y[k + 3 * M] = {b.x - g1 * dm.x, b.y - g1 * dm.y};
        } else {
            const cx<T> t3 = {g3 * v3.x, g3 * v3.y};
            c = {g1 * v1.x + t3.x, g1 * v1.y + t3.y};
            d = cmul_i<T, SIGN>(cx<T>{g1 * v1.x - t3.x, g1 * v1.y - t3.y});
            y[k] = cadd(a, c);
            y[k + 2 * M] = csub(a, c);
            y[k + M] = cadd(b, d);
            y[k + 3 * M] = csub(b, d);
        }
    } else {
        cx<T> u[R];
        sfor<R>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            u[r] = twiddle<T, SIGN, N, r * k>(sub[r][k]);
        });
        butterfly<T, R, SIGN>(u);
        sfor<R>([&](auto qI) {
            constexpr int q = decltype(qI)::value;
            y[k + M * q] = u[q];
        });
    }
}

// y[k] = sum_{m<N} x[OFF + IS*m] exp(SIGN 2 pi i m k / N), k = 0..N-1
template <typename T, int N, int SIGN, int IS, int OFF, int LEN>
FKS_HD void fft_rec(const cx<T> (&x)[LEN], cx<T>* y) {
    if constexpr (N == 1) {
        y[0] = x[OFF];
    } else {
        constexpr int R = first_radix<N>();
        constexpr int M = N / R;
        cx<T> sub[R][M];
        sfor<R>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            fft_rec<T, M, SIGN, IS * R, OFF + IS * r, LEN>(x, sub[r]);
        });
        sfor<M>([&](auto kI) {
            combine<T, N, SIGN, R, M, decltype(kI)::value>(sub, y);
        });
    }
}

// an empty asm that takes every value of v: the values exist at this point of the
// program, in registers, and the compiler does not move the code that computes
// them past the memory operations that follow
template <int K, typename T, int M>
FKS_HD void pin_from(cx<T> (&v)[M]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (K < M) {
        asm volatile("" : "+v"(v[K].x), "+v"(v[K].y) : : "memory");
        pin_from<K + 1>(v);
    }
#endif
}

// fft (below) with a hook: hook(I) runs after first-level sub-transform I (I < R) and
// after output group I - R of the last combination (R <= I < R + N/R), so that a
// caller can place independent work (LDS traffic, loads) between the transform's parts.
// The combination writes x in place (the sub-transforms have consumed the input), so
// after group k the outputs x[k + (N/R) q], q < R, are final and a hook may use them.
template <typename T, int N, int SIGN, typename Hook>
FKS_HD void fft_hook(cx<T> (&x)[N], Hook&& hook) {
    constexpr int R = first_radix<N>();
    constexpr int M = N / R;
    cx<T> sub[R][M];
    sfor<R>([&](auto rI) {
        constexpr int r = decltype(rI)::value;
        fft_rec<T, M, SIGN, R, r, N>(x, sub[r]);
        pin_from<0>(sub[r]);   // the sub-transform is finished here, not sunk past the hook's work
        hook(rI);
    });
    sfor<M>([&](auto kI) {
        constexpr int k = decltype(kI)::value;
        combine<T, N, SIGN, R, M, k>(sub, x);
        hook(std::integral_constant<int, R + k>{});
    });
}

template <typename T, int N, int SIGN>
FKS_HD void fft(cx<T> (&x)[N]) {
    cx<T> y[N];
    fft_rec<T, N, SIGN, 1, 0, N>(x, y);
    sfor<N>([&](auto kI) {
        constexpr int k = decltype(kI)::value;
        x[k] = y[k];
    });
}

}  // namespace fks
