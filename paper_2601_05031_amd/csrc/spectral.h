// Helpers shared by the spectral transforms (k_spectral.hip) and the tridiagonal solves and
// residual norms (k_solve.hip) of the Poisson problems.
#pragma once

#include "fft_reg.h"
#include "flow_check.h"
#include "vs_internal.h"

namespace vs {

namespace {

constexpr int kBlock = 256;

struct Ptr3 {
    double* p[3];
};
struct CPtr3 {
    const double* p[3];
};
// Pointers to the spectral intermediates, stored as ST (double, or float in the refined mode).
template <class ST>
struct SPtr3 {
    ST* p[3];
};
// Up to six components for the two-pass transforms: the vorticity and stream-vector fields of
// a step go through one launch per direction.
template <class ST>
struct SPtr6 {
    ST* p[6];
};
struct Ptr6 {
    double* p[6];
};

// Loads widen to double and stores narrow from double: inside a kernel all arithmetic is FP64.
__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }
__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ double2 ld2(const float* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
__device__ __forceinline__ void st2(float* p, double a, double b) {
    *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Arithmetic of the two-pass transforms follows the storage type ST of the spectral data:
// FP64 (double2 values) or, in the refined mode, FP32 (float2). Twiddles come from the FP64
// table, rounded to T.
template <class T>
using C2 = typename fftr::V2<T>::t;
template <class T>
__device__ __forceinline__ C2<T> mkc(T a, T b) {
    return fftr::V2<T>::mk(a, b);
}
typedef double tw2v __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ C2<T> cmul_tw(C2<T> a, tw2v w) {
    const T wr = (T)w.x, wi = (T)w.y;
    return mkc<T>(a.x * wr - a.y * wi, a.x * wi + a.y * wr);
}
// Two consecutive values of an ST array as a T pair; a T pair stored as ST.
template <class T>
__device__ __forceinline__ C2<T> ldc(const double* p) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    return mkc<T>((T)v.x, (T)v.y);
}
template <class T>
__device__ __forceinline__ C2<T> ldc(const float* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return mkc<T>((T)v.x, (T)v.y);
}
template <class T>
__device__ __forceinline__ void stc(double* p, T a, T b) {
    *reinterpret_cast<double2*>(p) = make_double2((double)a, (double)b);
}
template <class T>
__device__ __forceinline__ void stc(float* p, T a, T b) {
    *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
}
template <class T>
__device__ __forceinline__ T ldt(const double* p) { return (T)*p; }
template <class T>
__device__ __forceinline__ T ldt(const float* p) { return (T)*p; }

// Objects in global memory. Pointers that a batched launch reads from its device table are
// generic; typing the accesses through them as global keeps them global loads and stores
// (flat ones would also count against the LDS counter). Pairs go through clang's vector
// types, which have no constructors to object to the address space.
template <class T>
using Gl = __attribute__((address_space(1))) T;
typedef double gd2v __attribute__((ext_vector_type(2)));
typedef float gf2v __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ C2<T> ldc(const Gl<double>* p) {
    const gd2v v = *reinterpret_cast<const Gl<gd2v>*>(p);
    return mkc<T>((T)v.x, (T)v.y);
}
template <class T>
__device__ __forceinline__ C2<T> ldc(const Gl<float>* p) {
    const gf2v v = *reinterpret_cast<const Gl<gf2v>*>(p);
    return mkc<T>((T)v.x, (T)v.y);
}
template <class T>
__device__ __forceinline__ void stc(Gl<double>* p, T a, T b) {
    gd2v v;
    v.x = (double)a;
    v.y = (double)b;
    *reinterpret_cast<Gl<gd2v>*>(p) = v;
}
template <class T>
__device__ __forceinline__ void stc(Gl<float>* p, T a, T b) {
    gf2v v;
    v.x = (float)a;
    v.y = (float)b;
    *reinterpret_cast<Gl<gf2v>*>(p) = v;
}
template <class T>
__device__ __forceinline__ T ldt(const Gl<double>* p) { return (T)*p; }
template <class T>
__device__ __forceinline__ T ldt(const Gl<float>* p) { return (T)*p; }
// A pair of consecutive values as FP64.
__device__ __forceinline__ double2 ldg2(const Gl<double>* p) {
    const gd2v v = *reinterpret_cast<const Gl<gd2v>*>(p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 ldg2(const Gl<float>* p) {
    const gf2v v = *reinterpret_cast<const Gl<gf2v>*>(p);
    return make_double2((double)v.x, (double)v.y);
}

// The instance of a block and its index inside the instance: logical blocks are split into
// runs of nb per instance (see Over in vs_internal.h).
// A reference, not a copy: the structs hold small pointer arrays indexed by the block's
// component, and a local copy indexed at run time would live in scratch memory.
template <bool BATCH, class A>
__device__ __forceinline__ const A& inst_args(const A& one, const A* __restrict__ tab, int inst) {
    if constexpr (BATCH)
        return tab[inst];
    else
        return one;
}

// Element c (block-uniform) of a small array inside an argument struct, by a chain of
// selects: indexing it with a run-time c would move the struct to scratch memory and turn
// every load through the pointer into a flat access.
template <class P, int N>
__device__ __forceinline__ P pick(const P (&arr)[N], int c) {
    P r = arr[0];
#pragma unroll
    for (int q = 1; q < N; ++q) r = (c == q) ? arr[q] : r;
    return r;
}

// Component c of the right-hand side b at an interior node offset c0.
__device__ __forceinline__ double rhs_val(const RhsArgs& a, int c, int c0) {
    const double v = a.f[c][c0];
    return (a.mode == RHS_NEGW) ? -v : v;
}

// 7-point Laplacian at an interior node using the stored wall rows of u.
__device__ __forceinline__ double lap_interior(const double* __restrict__ u, const Dims& d, int i,
                                               int j, int k) {
    const int c0 = node(d, i, j, k);
    const int ip = (i + 1 == d.nx) ? 0 : i + 1;
    const int im = (i == 0) ? d.nx - 1 : i - 1;
    const int kp = (k + 1 == d.nz) ? 0 : k + 1;
    const int km = (k == 0) ? d.nz - 1 : k - 1;
    return (u[node(d, ip, j, k)] + u[node(d, im, j, k)] + u[c0 + d.nz] + u[c0 - d.nz] +
            u[c0 - k + kp] + u[c0 - k + km] - 6.0 * u[c0]) *
           d.inv_h2;
}

// Wall contribution of the Dirichlet values to row j (nonzero only for j = 1 and j = M).
__device__ __forceinline__ double wall_term(const double* __restrict__ u, const Dims& d, int i,
                                            int j, int k) {
    double w = 0.0;
    if (j == 1) w += u[node(d, i, 0, k)];
    if (j == d.M) w += u[node(d, i, d.ny - 1, k)];
    return w * d.inv_h2;
}

// Two-pass shape (B, A) for a line length, or (0, 0) if the LDS Stockham path is used.
void two_pass_shape(int n, int& B, int& A) {
    B = 16;
    switch (n) {
        case 32: B = 8; A = 4; return;
        case 48: A = 3; return;
        case 64: A = 4; return;
        case 96: A = 6; return;
        case 128: A = 8; return;
        case 192: A = 12; return;
        case 256: A = 16; return;
        default: B = 0; A = 0; return;
    }
}

#define VS_TWO_PASS_CASES(X) X(8, 4) X(16, 3) X(16, 4) X(16, 6) X(16, 8) X(16, 12) X(16, 16)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <class ST>
SPtr3<ST> sptr(void* const spec[3], int ncomp) {
    return SPtr3<ST>{{static_cast<ST*>(spec[0]), ncomp > 1 ? static_cast<ST*>(spec[1]) : nullptr,
                      ncomp > 2 ? static_cast<ST*>(spec[2]) : nullptr}};
}

}  // namespace
}  // namespace vs
