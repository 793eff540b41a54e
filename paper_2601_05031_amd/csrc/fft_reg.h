// In-register complex DFTs of small compile-time sizes (2, 3, 4, 6, 8, 12, 16), natural order
// in and out, forward sign exp(-2 pi i p k / R), in FP64 (double2) or FP32 (float2). Sizes 6, 8, 12, 16 are built by one
// Cooley-Tukey split R = R1 * R2 (input index k1 + R1 k2, output index p2 + R2 p1) with
// compile-time twiddles exp(-2 pi i k1 p2 / R).
#pragma once

#include <hip/hip_runtime.h>

namespace vs {
namespace fftr {

struct cd {
    double re, im;
};

// exp(-2 pi i m / 16) = cos(pi m / 8) - i sin(pi m / 8)
__host__ __device__ constexpr cd w16(int m) {
    constexpr double c1 = 0.92387953251128675613;   // cos(pi/8)
    constexpr double s1 = 0.38268343236508977173;   // sin(pi/8)
    constexpr double r2 = 0.70710678118654752440;   // cos(pi/4)
    switch (m & 15) {
        case 0: return {1.0, 0.0};
        case 1: return {c1, -s1};
        case 2: return {r2, -r2};
        case 3: return {s1, -c1};
        case 4: return {0.0, -1.0};
        case 5: return {-s1, -c1};
        case 6: return {-r2, -r2};
        case 7: return {-c1, -s1};
        case 8: return {-1.0, 0.0};
        case 9: return {-c1, s1};
        case 10: return {-r2, r2};
        case 11: return {-s1, c1};
        case 12: return {0.0, 1.0};
        case 13: return {s1, c1};
        case 14: return {r2, r2};
        default: return {c1, s1};
    }
}

// exp(-2 pi i m / 12) = cos(pi m / 6) - i sin(pi m / 6)
__host__ __device__ constexpr cd w12(int m) {
    constexpr double h3 = 0.86602540378443864676;   // sqrt(3)/2
    switch (m % 12) {
        case 0: return {1.0, 0.0};
        case 1: return {h3, -0.5};
        case 2: return {0.5, -h3};
        case 3: return {0.0, -1.0};
        case 4: return {-0.5, -h3};
        case 5: return {-h3, -0.5};
        case 6: return {-1.0, 0.0};
        case 7: return {-h3, 0.5};
        case 8: return {-0.5, h3};
        case 9: return {0.0, 1.0};
        case 10: return {0.5, h3};
        default: return {h3, 0.5};
    }
}

// exp(-2 pi i m / R) for R dividing 16 or 12.
__host__ __device__ constexpr cd wr(int R, int m) {
    return (16 % R == 0) ? w16((m % R) * (16 / R)) : w12((m % R) * (12 / R));
}

// Complex values as HIP's double2 or float2: the transforms run in the precision of the data
// they carry (FP64, or FP32 in the refined mode).
template <class T>
struct V2;
template <>
struct V2<double> {
    using t = double2;
    static __device__ __forceinline__ double2 mk(double a, double b) { return make_double2(a, b); }
};
template <>
struct V2<float> {
    using t = float2;
    static __device__ __forceinline__ float2 mk(float a, float b) { return make_float2(a, b); }
};

template <class C>
__device__ __forceinline__ C cadd(C a, C b) {
    C r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <class C>
__device__ __forceinline__ C csub(C a, C b) {
    C r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <class C>
__device__ __forceinline__ C cmulw(C a, cd w) {
    using T = decltype(a.x);
    const T wr_ = (T)w.re, wi = (T)w.im;
    C r;
    r.x = a.x * wr_ - a.y * wi;
    r.y = a.x * wi + a.y * wr_;
    return r;
}

template <int R>
struct DFT;

template <>
struct DFT<2> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) {
        const C a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <>
struct DFT<3> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) {
        using T = decltype(x[0].x);
        const T c = (T)0.86602540378443864676;
        const T half = (T)0.5;
        const C s = cadd(x[1], x[2]);
        const C e = csub(x[1], x[2]);
        C m;
        m.x = x[0].x - half * s.x;
        m.y = x[0].y - half * s.y;
        x[0] = cadd(x[0], s);
        x[1].x = m.x + c * e.y;
        x[1].y = m.y - c * e.x;
        x[2].x = m.x - c * e.y;
        x[2].y = m.y + c * e.x;
    }
};

template <>
struct DFT<4> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) {
        const C a = cadd(x[0], x[2]);
        const C b = csub(x[0], x[2]);
        const C c = cadd(x[1], x[3]);
        const C e = csub(x[1], x[3]);
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1].x = b.x + e.y;
        x[1].y = b.y - e.x;
        x[3].x = b.x - e.y;
        x[3].y = b.y + e.x;
    }
};

template <int R1, int R2, class C>
__device__ __forceinline__ void dft_split(C* x) {
    constexpr int R = R1 * R2;
    C y[R];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        C t[R2];
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) t[k2] = x[k1 + R1 * k2];
        DFT<R2>::run(t);
#pragma unroll
        for (int p2 = 0; p2 < R2; ++p2)
            y[k1 * R2 + p2] = ((k1 * p2) % R == 0) ? t[p2] : cmulw(t[p2], wr(R, k1 * p2));
    }
#pragma unroll
    for (int p2 = 0; p2 < R2; ++p2) {
        C t[R1];
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) t[k1] = y[k1 * R2 + p2];
        DFT<R1>::run(t);
#pragma unroll
        for (int p1 = 0; p1 < R1; ++p1) x[p2 + R2 * p1] = t[p1];
    }
}

template <>
struct DFT<6> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) { dft_split<2, 3>(x); }
};
template <>
struct DFT<8> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) { dft_split<2, 4>(x); }
};
template <>
struct DFT<12> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) { dft_split<4, 3>(x); }
};
template <>
struct DFT<16> {
    template <class C>
    static __device__ __forceinline__ void run(C* x) { dft_split<4, 4>(x); }
};

}  // namespace fftr
}  // namespace vs
