// Internal types shared by the gfx950 kernels: complex arithmetic, storage
// precisions and the internal field layouts.
//
// Internal spinor layout (one parity, "half field"): structure of 16-byte
// planes over the 12 spin-colour components c = spin*3 + colour,
//     data[q][i] = components (q*CPP .. q*CPP + CPP-1) of 5D site i,
//     i = j*Ls + s,  j the site's internal 4D index,  CPP = 16/sizeof(complex)
// so that the lanes of a wavefront, which walk i with s fastest, each load 16
// contiguous bytes of one plane.  FP16 fields carry one float scale per 5D
// site (norm[i] = max |re|,|im| over the site's 24 reals; data holds
// value/scale).
//
// Internal gauge layout: per output parity p and direction d = 0..7
// (+x,+y,+z,+t,-x,-y,-z,-t) the link the hop multiplies with, already
// conjugated for the backward directions:
//     link[p][d][k][cb], k = row*3 + col,  U_mu(x) for d < 4, U_mu(x-mu)^+ for d >= 4
// and the checkerboard index of the neighbour, nbr[p][d][cb].
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dwf {

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
// i*a and -i*a
template <typename T>
__host__ __device__ __forceinline__ cx<T> timesI(cx<T> a) { return {-a.im, a.re}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> timesMinusI(cx<T> a) { return {a.im, -a.re}; }
// acc += a*b
template <typename T>
__host__ __device__ __forceinline__ void cmac(cx<T> &acc, cx<T> a, cx<T> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// ------------------------------------------------------------ storage types

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

// epilogue kinds of the fused stencil
enum EpiKind { EPI_NONE = 0, EPI_DENSE = 1, EPI_SHIFT = 2, EPI_TOEP = 3 };

struct F64 {
    using elem = double2;
    using real = double;
    static constexpr bool has_norm = false;
    static constexpr int prec = P_F64;
};
struct F32 {
    using elem = float2;
    using real = float;
    static constexpr bool has_norm = false;
    static constexpr int prec = P_F32;
};
// The links of the 16-bit storage precisions (LinkQ15 below) are kept in 16-bit
// fixed point (value = integer / 32767; SU(3) entries are bounded by 1 in
// modulus), absolute error 1.5e-5 per entry against up to 2.4e-4 in FP16 and
// 2e-3 in BF16.  A perturbed link changes the low-precision operator itself,
// by an amount that is large against its smallest eigenvalues on lattices
// with light modes; the spinor fields keep the floating-point formats.
struct F16 {
    using elem = __half2;
    using real = float;
    static constexpr bool has_norm = true;
    static constexpr int prec = P_F16;
};
struct BF16 {
    using elem = __hip_bfloat162;
    using real = float;
    static constexpr bool has_norm = false;
    static constexpr int prec = P_BF16;
};

// 16-bit fixed-point link entry pair (re, im), as stored by the 16-bit precisions
__host__ __device__ __forceinline__ uint32_t pack_q15(double re, double im)
{
    auto q = [](double v) -> uint32_t {
        double t = v * 32767.0;
        t = t > 32767.0 ? 32767.0 : (t < -32767.0 ? -32767.0 : t);
        const int k = (int)(t >= 0 ? t + 0.5 : t - 0.5);
        return (uint32_t)(uint16_t)(int16_t)k;
    };
    return q(re) | (q(im) << 16);
}
template <typename C>
__device__ __forceinline__ cx<C> unpack_q15(uint32_t w)
{
    const C k = C(1.0 / 32767.0);
    return {k * C((int16_t)(w & 0xffffu)), k * C((int16_t)(w >> 16))};
}
template <typename S>
struct LinkQ15 {
    static constexpr bool value = false;
};
template <>
struct LinkQ15<F16> {
    static constexpr bool value = true;
};
template <>
struct LinkQ15<BF16> {
    static constexpr bool value = true;
};

template <typename C>
__device__ __forceinline__ cx<C> unpack(double2 v) { return {C(v.x), C(v.y)}; }
template <typename C>
__device__ __forceinline__ cx<C> unpack(float2 v) { return {C(v.x), C(v.y)}; }
template <typename C>
__device__ __forceinline__ cx<C> unpack(__half2 v)
{
    float2 f = __half22float2(v);
    return {C(f.x), C(f.y)};
}
template <typename C>
__device__ __forceinline__ cx<C> unpack(__hip_bfloat162 v)
{
    float2 f = __bfloat1622float2(v);
    return {C(f.x), C(f.y)};
}

template <typename S, typename C>
__device__ __forceinline__ typename S::elem pack(cx<C> v);
template <>
__device__ __forceinline__ double2 pack<F64, double>(cx<double> v) { return make_double2(v.re, v.im); }
template <>
__device__ __forceinline__ double2 pack<F64, float>(cx<float> v) { return make_double2(v.re, v.im); }
template <>
__device__ __forceinline__ float2 pack<F32, float>(cx<float> v) { return make_float2(v.re, v.im); }
template <>
__device__ __forceinline__ float2 pack<F32, double>(cx<double> v) { return make_float2(float(v.re), float(v.im)); }
template <>
__device__ __forceinline__ __half2 pack<F16, float>(cx<float> v) { return __float22half2_rn(make_float2(v.re, v.im)); }
template <>
__device__ __forceinline__ __half2 pack<F16, double>(cx<double> v)
{
    return __float22half2_rn(make_float2(float(v.re), float(v.im)));
}
template <>
__device__ __forceinline__ __hip_bfloat162 pack<BF16, float>(cx<float> v)
{
    return __float22bfloat162_rn(make_float2(v.re, v.im));
}
template <>
__device__ __forceinline__ __hip_bfloat162 pack<BF16, double>(cx<double> v)
{
    return __float22bfloat162_rn(make_float2(float(v.re), float(v.im)));
}

// A half field in internal layout: 12 component planes of n 5D sites.
struct Field {
    void *data;
    float *norm;  // FP16 only
    long n;       // 5D sites in the field (Vh * Ls)
};

// Spinor planes are 16 bytes wide: plane q of site i holds the CPP = 16 /
// sizeof(elem) consecutive components CPP*q .. CPP*q + CPP - 1, so that one
// lane moves 16 bytes per load and a wavefront 1 KiB of one plane.
template <typename S>
struct Planes {
    static constexpr int cpp = 16 / sizeof(typename S::elem);  // components per plane
    static constexpr int n = 12 / cpp;                           // planes per spinor
};

union Vec16 {
    uint4 u;
    double2 d[1];
    float2 f[2];
    __half2 h[4];
    __hip_bfloat162 b[4];
};

template <typename S>
__device__ __forceinline__ typename S::elem vec_get(const Vec16 &v, int k)
{
    if constexpr (sizeof(typename S::elem) == 16) return v.d[0];
    else if constexpr (sizeof(typename S::elem) == 8) return v.f[k];
    else if constexpr (S::prec == P_F16) return v.h[k];
    else return v.b[k];
}

template <typename S>
__device__ __forceinline__ void vec_set(Vec16 &v, int k, typename S::elem e)
{
    if constexpr (sizeof(typename S::elem) == 16) v.d[0] = e;
    else if constexpr (sizeof(typename S::elem) == 8) v.f[k] = e;
    else if constexpr (S::prec == P_F16) v.h[k] = e;
    else v.b[k] = e;
}

template <typename S, typename C>
__device__ __forceinline__ void load_spinor(const Field &f, long i, cx<C> v[12])
{
    using P = Planes<S>;
    const uint4 *d = (const uint4 *)f.data;
    C scale = C(1);
    if constexpr (S::has_norm) scale = C(f.norm[i]);
#pragma unroll
    for (int q = 0; q < P::n; q++) {
        Vec16 w;
        w.u = d[q * f.n + i];
#pragma unroll
        for (int k = 0; k < P::cpp; k++) {
            cx<C> t = unpack<C>(vec_get<S>(w, k));
            if constexpr (S::has_norm) t = scale * t;
            v[q * P::cpp + k] = t;
        }
    }
}

// the stored components without the FP16 site scale, and the scale (1 for
// formats without one); value = scale * v
template <typename S, typename C>
__device__ __forceinline__ void load_spinor_unscaled(const Field &f, long i, cx<C> v[12], C &scale)
{
    using P = Planes<S>;
    const uint4 *d = (const uint4 *)f.data;
    scale = C(1);
    if constexpr (S::has_norm) scale = C(f.norm[i]);
#pragma unroll
    for (int q = 0; q < P::n; q++) {
        Vec16 w;
        w.u = d[q * f.n + i];
#pragma unroll
        for (int k = 0; k < P::cpp; k++) v[q * P::cpp + k] = unpack<C>(vec_get<S>(w, k));
    }
}

// a spinor as stored (planes and scale), to be unpacked later; lets a kernel
// issue the load early without holding the unpacked components
template <typename S>
struct RawSpinor {
    uint4 q[Planes<S>::n];
    float norm;
};

template <typename S>
__device__ __forceinline__ void load_raw(const Field &f, long i, RawSpinor<S> &r)
{
    using P = Planes<S>;
    const uint4 *d = (const uint4 *)f.data;
#pragma unroll
    for (int q = 0; q < P::n; q++) r.q[q] = d[q * f.n + i];
    r.norm = S::has_norm ? f.norm[i] : 1.f;
}

template <typename S, typename C>
__device__ __forceinline__ void unpack_raw(const RawSpinor<S> &r, cx<C> v[12])
{
    using P = Planes<S>;
    const C scale = C(r.norm);
#pragma unroll
    for (int q = 0; q < P::n; q++) {
        Vec16 w;
        w.u = r.q[q];
#pragma unroll
        for (int k = 0; k < P::cpp; k++) {
            cx<C> t = unpack<C>(vec_get<S>(w, k));
            if constexpr (S::has_norm) t = scale * t;
            v[q * P::cpp + k] = t;
        }
    }
}

// NT: non-temporal stores, for outputs that the writing kernel does not read
// again (they are not kept in the caches at the expense of its inputs)
template <typename S, typename C, bool NT = false>
__device__ __forceinline__ void store_spinor(const Field &f, long i, const cx<C> v[12])
{
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    using P = Planes<S>;
    uint4 *d = (uint4 *)f.data;
    C inv = C(1);
    if constexpr (S::has_norm) {
        C m = C(0);
#pragma unroll
        for (int c = 0; c < 12; c++) m = fmax(m, fmax(fabs(v[c].re), fabs(v[c].im)));
        inv = (m > C(0)) ? C(1) / m : C(0);
        if constexpr (NT) __builtin_nontemporal_store(float(m), f.norm + i);
        else f.norm[i] = float(m);
    }
#pragma unroll
    for (int q = 0; q < P::n; q++) {
        Vec16 w;
#pragma unroll
        for (int k = 0; k < P::cpp; k++) {
            const cx<C> t = S::has_norm ? inv * v[q * P::cpp + k] : v[q * P::cpp + k];
            vec_set<S>(w, k, pack<S, C>(t));
        }
        if constexpr (NT) __builtin_nontemporal_store(__builtin_bit_cast(v4u, w.u), (v4u *)(d + q * f.n + i));
        else d[q * f.n + i] = w.u;
    }
}

// v becomes the value that store_spinor followed by load_spinor returns: the
// storage rounding (and the FP16 site scale) applied in registers.  A kernel
// that stores a field and also uses its values further (the A p of the CG
// direction, the norm of the updated residual) uses the rounded values, so
// that what it computes is consistent with the stored field.
template <typename S, typename C>
__device__ __forceinline__ void storage_round(cx<C> v[12])
{
    if constexpr (S::has_norm) {
        C m = C(0);
#pragma unroll
        for (int c = 0; c < 12; c++) m = fmax(m, fmax(fabs(v[c].re), fabs(v[c].im)));
        const C inv = (m > C(0)) ? C(1) / m : C(0);
        const C scale = C(float(m));
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = scale * unpack<C>(pack<S, C>(inv * v[c]));
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = unpack<C>(pack<S, C>(v[c]));
    }
}

// Value of (P5 psi) (dag = false) or (P5^+ psi) (dag = true) at slice s for
// spin-colour component c, read from the Ls x 12 block of one 4D site:
//   P5 psi_s = P_- psi_{s+1} + P_+ psi_{s-1},  P5^+ psi_s = P_+ psi_{s+1} + P_- psi_{s-1},
// with psi_Ls = -mf psi_0 and psi_-1 = -mf psi_{Ls-1}.  Components c < 6 are
// the P_+ spins (0, 1), c >= 6 the P_- spins (2, 3).
template <typename C>
__device__ __forceinline__ cx<C> shift5(const cx<C> *blk, int c, int s, int Ls, bool dag, C mf)
{
    const bool up = c < 6;
    int src = (up != dag) ? s - 1 : s + 1;
    C f = C(1);
    if (src < 0) {
        src = Ls - 1;
        f = -mf;
    } else if (src >= Ls) {
        src = 0;
        f = -mf;
    }
    return f * blk[src * 12 + c];
}

// the same, with the block laid out component-major: rows[c * Ls + s]
// (consecutive lanes s touch consecutive words: no LDS bank conflicts)
template <typename C>
__device__ __forceinline__ cx<C> shift5t(const cx<C> *rows, int c, int s, int Ls, bool dag, C mf)
{
    const bool up = c < 6;
    int src = (up != dag) ? s - 1 : s + 1;
    C f = C(1);
    if (src < 0) {
        src = Ls - 1;
        f = -mf;
    } else if (src >= Ls) {
        src = 0;
        f = -mf;
    }
    return f * rows[c * Ls + src];
}

// Sum of v over the workgroup (fixed order: wavefront tree, then waves in
// order); the result is valid in thread 0.  Every thread must call it.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wave = tid >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0;
    if (tid == 0)
        for (int w = 0; w < nw; w++) t += red[w];
    __syncthreads();
    return t;
}

// Workgroup -> tile mapping that keeps each XCD on contiguous runs of `run`
// tiles.  Workgroups are dealt to the 8 XCDs round-robin; without the remap
// neighbouring tiles land in different L2 caches.  Bijective on [0, nblk).
__device__ __forceinline__ int xcd_swizzle(int b, int nblk, int run)
{
    if (run <= 1) return b;
    const int chunk = 8 * run;
    const int full = (nblk / chunk) * chunk;
    if (b >= full) return b;
    const int k = b >> 3, x = b & 7;
    return (k / run) * chunk + x * run + (k % run);
}

}  // namespace dwf
