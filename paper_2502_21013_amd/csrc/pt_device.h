// Device-side helpers: slot arithmetic, stencil access, workgroup mapping.
#pragma once

#include <hip/hip_runtime.h>

#include "pt_internal.h"

namespace pt {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T> __device__ __forceinline__ typename Vec2<T>::type mk2(T x, T y) {
    typename Vec2<T>::type r;
    r.x = x;
    r.y = y;
    return r;
}

// Generic per-slot scalar in (a, b, c) form (see pt_internal.h).
template <typename T> struct GS {
    T a, b, c;
};

template <typename T> __device__ __forceinline__ GS<T> gs_from(double2 v, bool s0) {
    GS<T> g;
    g.a = (T)v.x;
    g.b = s0 ? (T)0 : (T)v.y;
    g.c = s0 ? (T)v.y : (T)v.x;
    return g;
}

template <typename T, typename T2> __device__ __forceinline__ T2 gs_apply(const GS<T>& g, T2 w) {
    T2 r;
    r.x = g.a * w.x - g.b * w.y;
    r.y = g.c * w.y + g.b * w.x;
    return r;
}

// Reciprocal of a positive number: hardware estimate (float), or the estimate refined by
// two Newton steps r <- r + r (1 - x r) (double, full precision).
template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// gs_inv_diag without a branch: both forms computed, the dm = 0 one selected (same values).
template <typename T> __device__ __forceinline__ GS<T> gs_inv_diag_sel(T dl, T idl, T dm, const GS<T>& z) {
    const T P = dl + z.a * dm, Pp = dl + z.c * dm, Q = z.b * dm;
    const T inv = fast_rcp<T>(P * Pp + Q * Q);
    const bool zero = dm == (T)0;
    GS<T> g;
    g.a = zero ? idl : Pp * inv;
    g.b = zero ? (T)0 : -Q * inv;
    g.c = zero ? idl : P * inv;
    return g;
}

// Inverse of D = dl + z (x) dm (z generic, dl > 0 and dm >= 0 real), in generic form;
// idl = 1/dl is the inverse where dm = 0 (no conductivity near the node).
template <typename T> __device__ __forceinline__ GS<T> gs_inv_diag(T dl, T idl, T dm, const GS<T>& z) {
    GS<T> g;
    if (dm == (T)0) {
        g.a = idl;
        g.b = (T)0;
        g.c = idl;
        return g;
    }
    T P = dl + z.a * dm;   // acts on .x
    T Pp = dl + z.c * dm;  // acts on .y
    T Q = z.b * dm;
    T inv = fast_rcp<T>(P * Pp + Q * Q);
    g.a = Pp * inv;
    g.b = -Q * inv;
    g.c = P * inv;
    return g;
}

template <typename T2> __device__ __forceinline__ T2 add2(T2 a, T2 b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <typename T2> __device__ __forceinline__ T2 sub2(T2 a, T2 b) {
    a.x -= b.x;
    a.y -= b.y;
    return a;
}
template <typename T, typename T2> __device__ __forceinline__ T2 scale2(T s, T2 a) {
    a.x *= s;
    a.y *= s;
    return a;
}
template <typename T, typename T2> __device__ __forceinline__ T2 fma2(T s, T2 a, T2 acc) {
    acc.x += s * a.x;
    acc.y += s * a.y;
    return acc;
}
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
    T2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T2> __device__ __forceinline__ T2 conj2(T2 a) {
    a.y = -a.y;
    return a;
}
// multiply by -i
template <typename T2> __device__ __forceinline__ T2 mul_mi(T2 a) {
    T2 r;
    r.x = a.y;
    r.y = -a.x;
    return r;
}

// Accumulate the three partial sums of a slot dot product:
//   s1 += u.x v.x,  s2 += u.y v.y,  s3 += u.x v.y -/+ u.y v.x
// conj = true gives the Hermitian form u^H v, false the bilinear form u^T v.
template <typename T2> __device__ __forceinline__ void dot3_acc(double* s, T2 u, T2 v, bool conj) {
    s[0] += (double)u.x * (double)v.x;
    s[1] += (double)u.y * (double)v.y;
    double cr = (double)u.x * (double)v.y;
    double rc = (double)u.y * (double)v.x;
    s[2] += conj ? (cr - rc) : (cr + rc);
}

// Column and row range of this workgroup in a sweeping kernel (see Geom).
struct SweepRange {
    int col0, row0, row1;
};

// (also compiled for the host: the launch-bounds check walks the same ranges)
__host__ __device__ __forceinline__ SweepRange sweep_range(int vb, int col_groups, int per_step, int rows_per_chunk,
                                                           int side) {
    SweepRange r;
    int g = vb % col_groups, c = vb / col_groups;
    r.col0 = g * per_step;
    r.row0 = c * rows_per_chunk;
    r.row1 = r.row0 + rows_per_chunk < side ? r.row0 + rows_per_chunk : side;
    if (r.row0 > side) r.row0 = side;
    return r;
}

// Virtual workgroup index of workgroup b of a launch of `blocks` workgroups: workgroups are
// dispatched round-robin over the XCDs, so this gives every XCD a contiguous range of node
// groups (its own L2 sees the stencil neighbours of what it processes). blocks is a multiple of
// kNumXcd. virtual_block is the same for the calling workgroup.
__host__ __device__ __forceinline__ int virtual_block_of(int b, int blocks, int remap) {
    if (!remap) return b;
    const int per = blocks / kNumXcd;
    return (b % kNumXcd) * per + b / kNumXcd;
}
__device__ __forceinline__ int virtual_block(int remap) { return virtual_block_of(blockIdx.x, gridDim.x, remap); }

// Read-only table entry at an index that is the same on every lane of the wavefront (UNI):
// read through the scalar unit (constant address space), so that the wait for it does not
// also wait for the vector loads in flight. The tables (materials, mass, load) are never
// written while a kernel reads them, and the scalar data cache is invalidated at every
// kernel launch, so it needs no coherence with the vector stores.
template <typename X> using ConstPtr = const __attribute__((address_space(4))) X*;

template <bool UNI, typename X>
__device__ __forceinline__ X uload(const X* p, size_t idx) {
    if constexpr (UNI) return ((ConstPtr<X>)p)[idx];
    else return p[idx];
}

// Compiler-only ordering point: memory operations are not moved across it (no instruction
// is emitted). Placed after a prefetch so that the loads are issued before the arithmetic
// that precedes their first use instead of being sunk next to it.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// Marks a loaded value as used here on every path (no instruction is emitted): the wait for
// the load then sits at this point on all paths, instead of a conservative wait for all
// loads at a later register reuse on paths where the value is never read.
__device__ __forceinline__ void consume(double x) { asm volatile("" ::"v"(x)); }
__device__ __forceinline__ void consume(float x) { asm volatile("" ::"v"(x)); }
__device__ __forceinline__ void consume(double2 x) {
    consume(x.x);
    consume(x.y);
}
__device__ __forceinline__ void consume(float2 x) {
    consume(x.x);
    consume(x.y);
}

// Nonzero test on the raw bits (x != 0 exactly when the bits without the sign are nonzero,
// NaN included): OR-ing several of them keeps a test of wave-uniform values on the scalar unit
// instead of one vector compare per value.
__device__ __forceinline__ unsigned long long nzbits(double x) { return __builtin_bit_cast(unsigned long long, x) << 1; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Streaming (nontemporal) access for data touched once per sweep and far larger than the
// caches: the lines are not kept in L2 / MALL at the expense of data that is reused (the
// neighbour columns of the stencil sweeps). X is moved as 16-byte pieces.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
template <typename X>
__device__ __forceinline__ X nt_load(const X* p) {
    static_assert(sizeof(X) % 16 == 0, "moved in 16-byte pieces");
    X x;
    nt_f4* d = (nt_f4*)&x;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(X) / 16); ++k) d[k] = __builtin_nontemporal_load((const nt_f4*)p + k);
    return x;
}
template <typename X>
__device__ __forceinline__ void nt_store(X* p, const X& x) {
    static_assert(sizeof(X) % 16 == 0, "moved in 16-byte pieces");
    const nt_f4* s = (const nt_f4*)&x;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(X) / 16); ++k) __builtin_nontemporal_store(s[k], (nt_f4*)p + k);
}

// ---------------------------------------------------------------- reluctivity laws (Sec. 4)

// Law of one region, parameters q = (q.x, q.y, q.z, q.w), before the triangle's scale theta:
//   PT_NU_RATIONAL  nu = q.x + q.y s^2 / (1 + s^2)
//   PT_NU_EXPCAP    nu = q.x exp(q.y min(s^2, q.z)) + q.w, q.z = ln(c)/b: a min(exp(b s^2), c) + d
//                   (q.z huge when b = 0, the constant a + d)
// with s^2 = |grad u|^2. law_nu_dn also gives dnu/d(s^2): q.y / (1+s^2)^2, resp. a b exp(b s^2)
// below the saturation kink and 0 from it on (the right derivative).
template <int LAW> __device__ __forceinline__ double law_nu(const double4 q, double s2) {
    if constexpr (LAW == PT_NU_RATIONAL) return (q.x + q.y) - q.y / (1.0 + s2);
    else return q.x * exp(q.y * fmin(s2, q.z)) + q.w;
}

template <int LAW> __device__ __forceinline__ double law_nu_dn(const double4 q, double s2, double& dn) {
    if constexpr (LAW == PT_NU_RATIONAL) {
        const double r = fast_rcp<double>(1.0 + s2);
        dn = q.y * r * r;
        return (q.x + q.y) - q.y * r;
    } else {
        const double e = exp(q.y * fmin(s2, q.z));
        dn = s2 < q.z ? q.x * q.y * e : 0.0;
        return q.x * e + q.w;
    }
}

}  // namespace pt
