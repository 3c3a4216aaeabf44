// Vector kernels: reductions with deterministic FP64 accumulation, linear
// combinations, precision conversions and the fused conjugate-gradient updates.
// One lane per 5D site (12 complex components); scalars that the Krylov loops
// produce on the device are read from device memory so no host round trip sits
// between dependent kernels.
#include "dwf_internal.h"

namespace dwf {

static constexpr int BS = 256;

static dim3 g1(long n) { return dim3((unsigned)((n + BS - 1) / BS)); }

#define DWF_DISPATCH(prec, KERNEL, grid, blk, lds, ...)                                                    \
    switch (prec) {                                                                                        \
    case P_F64: hipLaunchKernelGGL(KERNEL<F64>, grid, blk, lds, c.stream, __VA_ARGS__); break;             \
    case P_F32: hipLaunchKernelGGL(KERNEL<F32>, grid, blk, lds, c.stream, __VA_ARGS__); break;             \
    case P_F16: hipLaunchKernelGGL(KERNEL<F16>, grid, blk, lds, c.stream, __VA_ARGS__); break;             \
    default: hipLaunchKernelGGL(KERNEL<BF16>, grid, blk, lds, c.stream, __VA_ARGS__); break;               \
    }                                                                                                      \
    HIPCHECK(hipGetLastError())

template <typename S>
using Cof = typename S::real;

template <typename S>
__global__ void __launch_bounds__(BS) k_norm2(Field a, double *partial)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double t = 0;
    if (i < a.n) {
        cx<C> v[12];
        load_spinor<S, C>(a, i, v);
        for (int c = 0; c < 12; c++) t += double(v[c].re) * double(v[c].re) + double(v[c].im) * double(v[c].im);
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// <a, b> = sum conj(a) b
template <typename S>
__global__ void __launch_bounds__(BS) k_dot(Field a, Field b, double *partial)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double re = 0, im = 0;
    if (i < a.n) {
        cx<C> u[12], v[12];
        load_spinor<S, C>(a, i, u);
        load_spinor<S, C>(b, i, v);
        for (int c = 0; c < 12; c++) {
            re += double(u[c].re) * double(v[c].re) + double(u[c].im) * double(v[c].im);
            im += double(u[c].re) * double(v[c].im) - double(u[c].im) * double(v[c].re);
        }
    }
    re = block_sum(re);
    im = block_sum(im);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = re;
        partial[2 * blockIdx.x + 1] = im;
    }
}

// fixed-order sum of nparts partials of `width` doubles -> dscal[slot + w].
// One workgroup of FBS threads; thread t sums partials t, t + FBS, ... in four
// interleaved running sums, so the order depends only on nparts.
static constexpr int FBS = 1024;
// When mirror is set, the sums are also written there: host memory that the
// host reads after an event behind this kernel.  With qslot >= 0 (width 1) the
// quotient dscal[qslot] = dscal[nslot] / sum follows.
__global__ void __launch_bounds__(FBS) k_finish(const double *partial, int nparts, int width, double *dscal, int slot,
                                                double *mirror, int qslot, int nslot)
{
    for (int w = 0; w < width; w++) {
        double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        int k = threadIdx.x;
        for (; k + 3 * FBS < nparts; k += 4 * FBS) {
            t0 += partial[(long)k * width + w];
            t1 += partial[(long)(k + FBS) * width + w];
            t2 += partial[(long)(k + 2 * FBS) * width + w];
            t3 += partial[(long)(k + 3 * FBS) * width + w];
        }
        for (; k < nparts; k += FBS) t0 += partial[(long)k * width + w];
        const double t = block_sum((t0 + t1) + (t2 + t3));
        if (threadIdx.x == 0) {
            dscal[slot + w] = t;
            if (mirror) mirror[w] = t;
            if (qslot >= 0 && w == 0) dscal[qslot] = dscal[nslot] / t;
        }
    }
}

__global__ void k_scalar_div(double *dscal, int out, int num, int den)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dscal[out] = dscal[num] / dscal[den];
}

// dscal[slot] = v, the value passed by argument: stream-ordered, no host wait
__global__ void k_set_scalar(double *dscal, int slot, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dscal[slot] = v;
}

// CG step scalars: beta = rho_new / rho, then rho = rho_new
__global__ void k_cg_beta(double *dscal, int beta, int rho, int rho_new)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double rn = dscal[rho_new];
        dscal[beta] = rn / dscal[rho];
        dscal[rho] = rn;
    }
}

template <typename S>
__global__ void __launch_bounds__(BS) k_axpby(double a, Field x, double b, Field y, Field z)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= x.n) return;
    cx<C> u[12], v[12];
    load_spinor<S, C>(x, i, u);
    load_spinor<S, C>(y, i, v);
    for (int c = 0; c < 12; c++) u[c] = C(a) * u[c] + C(b) * v[c];
    store_spinor<S, C>(z, i, u);
}

// z = a x + b y + c w (z may alias any input)
template <typename S>
__global__ void __launch_bounds__(BS) k_axpbypcz(double a, Field x, double b, Field y, double c, Field w, Field z)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= x.n) return;
    cx<C> u[12], v[12], t[12];
    load_spinor<S, C>(x, i, u);
    load_spinor<S, C>(y, i, v);
    load_spinor<S, C>(w, i, t);
    for (int k = 0; k < 12; k++) u[k] = C(a) * u[k] + C(b) * v[k] + C(c) * t[k];
    store_spinor<S, C>(z, i, u);
}

template <typename S>
__global__ void __launch_bounds__(BS) k_caxpy(double are, double aim, Field x, Field y)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= x.n) return;
    cx<C> u[12], v[12];
    load_spinor<S, C>(x, i, u);
    load_spinor<S, C>(y, i, v);
    const cx<C> a = mk(C(are), C(aim));
    for (int c = 0; c < 12; c++) cmac(v[c], a, u[c]);
    store_spinor<S, C>(y, i, v);
}

template <typename S>
__global__ void __launch_bounds__(BS) k_zero(Field a)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= a.n) return;
    cx<C> v[12];
    for (int c = 0; c < 12; c++) v[c] = mk(C(0), C(0));
    store_spinor<S, C>(a, i, v);
}

template <typename S>
__global__ void __launch_bounds__(BS) k_copy(Field a, Field b)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= a.n) return;
    cx<C> v[12];
    load_spinor<S, C>(a, i, v);
    store_spinor<S, C>(b, i, v);
}

// x += alpha p ; r -= alpha ap ; partial |r|^2.  x is kept in SX, which is
// wider than S for the 16-bit formats: the solution accumulates many
// increments and its rounding error is amplified by the condition number.
template <typename S, typename SX>
__global__ void __launch_bounds__(BS) k_cg_update_xr(Field x, Field r, Field p, Field ap, const double *dscal, int ia,
                                                      double *partial)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    const C alpha = C(dscal[ia]);
    double t = 0;
    if (i < x.n) {
        cx<C> xv[12], pv[12];
        load_spinor<SX, C>(x, i, xv);
        load_spinor<S, C>(p, i, pv);
        for (int c = 0; c < 12; c++) xv[c] = xv[c] + alpha * pv[c];
        store_spinor<SX, C>(x, i, xv);
        cx<C> rv[12], av[12];
        load_spinor<S, C>(r, i, rv);
        load_spinor<S, C>(ap, i, av);
        for (int c = 0; c < 12; c++) {
            rv[c] = rv[c] - alpha * av[c];
            t += double(rv[c].re) * double(rv[c].re) + double(rv[c].im) * double(rv[c].im);
        }
        store_spinor<S, C>(r, i, rv);
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// pout = r + beta p ; pa = (b + c P5) pout   (workgroup = Ls x sb lanes, one 4D
// site per row).  With ia >= 0 the pending solution updates are folded in
// first, x in storage precision SX: x += alpha_j q_j over the older directions
// of `older` (oldest first, alpha_j = dscal[slot_j]), then x += alpha p (alpha =
// dscal[ia], the old p).  pout may be p or an older direction: every lane reads
// its elements before it writes them.
template <typename S, typename SX>
__global__ void __launch_bounds__(256) k_cg_update_p(Field r, Field p, Field pout, Field pa, Field x, CgOlder older,
                                                     const double *dscal, int ib, int ia, long vh, int Ls, double bb,
                                                     double cc, double mf)
{
    using C = Cof<S>;
    const int s = threadIdx.x, j = threadIdx.y, sb = blockDim.y;
    const long cb = (long)blockIdx.x * sb + j;
    const bool valid = cb < vh;
    const long i = cb * Ls + s;
    const C beta = C(dscal[ib]);
    extern __shared__ unsigned char smem[];
    cx<C> *lds = (cx<C> *)smem;
    cx<C> pv[12];
    if (valid) {
        cx<C> rv[12];
        load_spinor<S, C>(p, i, pv);
        if (ia >= 0) {
            const C alpha = C(dscal[ia]);
            cx<C> xv[12];
            load_spinor<SX, C>(x, i, xv);
            for (int q = 0; q < older.n; q++) {
                const C alpha2 = C(dscal[older.slot[q]]);
                cx<C> qv[12];
                load_spinor<S, C>(older.dir[q], i, qv);
                for (int c = 0; c < 12; c++) xv[c] = xv[c] + alpha2 * qv[c];
            }
            for (int c = 0; c < 12; c++) xv[c] = xv[c] + alpha * pv[c];
            store_spinor<SX, C>(x, i, xv);
        }
        load_spinor<S, C>(r, i, rv);
        for (int c = 0; c < 12; c++) pv[c] = rv[c] + beta * pv[c];
        store_spinor<S, C>(pout, i, pv);
        // A is applied to the direction as stored: the operator then sees the
        // same vector in its hop terms (through pa) as in its diagonal terms
        // (through pout), and the solution update uses that vector too
        storage_round<S, C>(pv);
    } else {
        for (int c = 0; c < 12; c++) pv[c] = mk(C(0), C(0));
    }
    for (int c = 0; c < 12; c++) lds[(j * Ls + s) * 12 + c] = pv[c];
    __syncthreads();
    if (!valid) return;
    const cx<C> *blk = lds + j * Ls * 12;
    cx<C> out[12];
    for (int c = 0; c < 12; c++) out[c] = C(bb) * pv[c] + C(cc) * shift5<C>(blk, c, s, Ls, false, C(mf));
    store_spinor<S, C>(pa, i, out);
}

// x += alpha p with alpha = dscal[ia]; x in storage precision SX
template <typename S, typename SX>
__global__ void __launch_bounds__(BS) k_axpy_dev(Field x, Field p, const double *dscal, int ia)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= x.n) return;
    const C alpha = C(dscal[ia]);
    cx<C> xv[12], pv[12];
    load_spinor<SX, C>(x, i, xv);
    load_spinor<S, C>(p, i, pv);
    for (int c = 0; c < 12; c++) xv[c] = xv[c] + alpha * pv[c];
    store_spinor<SX, C>(x, i, xv);
}

// r = b - ax in FP64 ; partial |r|^2
__global__ void __launch_bounds__(BS) k_residual(Field b, Field ax, Field r, double *partial)
{
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double t = 0;
    if (i < b.n) {
        cx<double> u[12], v[12];
        load_spinor<F64, double>(b, i, u);
        load_spinor<F64, double>(ax, i, v);
        for (int c = 0; c < 12; c++) {
            u[c] = u[c] - v[c];
            t += u[c].re * u[c].re + u[c].im * u[c].im;
        }
        store_spinor<F64, double>(r, i, u);
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// xh += xl ; xl = 0
template <typename S>
__global__ void __launch_bounds__(BS) k_accumulate_low(Field xh, Field xl)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= xh.n) return;
    cx<double> h[12];
    cx<C> l[12];
    load_spinor<F64, double>(xh, i, h);
    load_spinor<S, C>(xl, i, l);
    for (int c = 0; c < 12; c++) {
        h[c] = h[c] + mk(double(l[c].re), double(l[c].im));
        l[c] = mk(C(0), C(0));
    }
    store_spinor<F64, double>(xh, i, h);
    store_spinor<S, C>(xl, i, l);
}

// multi-shift update for every active shift k:
//   x_k += a_k p_k ; p_k = z_k r + b_k p_k      coef[4k..4k+3] = (a_k, z_k, b_k, active)
template <typename S>
__global__ void __launch_bounds__(BS) k_ms_update(int nshift, const Field *x, const Field *p, Field r,
                                                   const double *coef)
{
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= r.n) return;
    cx<C> rv[12];
    load_spinor<S, C>(r, i, rv);
    for (int k = 0; k < nshift; k++) {
        if (coef[4 * k + 3] == 0.0) continue;
        const C a = C(coef[4 * k]), z = C(coef[4 * k + 1]), b = C(coef[4 * k + 2]);
        cx<C> xv[12], pv[12];
        load_spinor<S, C>(x[k], i, xv);
        load_spinor<S, C>(p[k], i, pv);
        for (int c = 0; c < 12; c++) {
            xv[c] = xv[c] + a * pv[c];
            pv[c] = z * rv[c] + b * pv[c];
        }
        store_spinor<S, C>(x[k], i, xv);
        store_spinor<S, C>(p[k], i, pv);
    }
}

// ------------------------------------------------ batched multi-shift CG
//
// All right-hand sides j advance together; shift k of rhs j is batch member
// k*nrhs + j of the solution and direction batches.  The shifted recurrences
// (Jegerlehner) run on the device, one workgroup per right-hand side:
//   zeta_{n+1} = zeta_n zeta_{n-1} a_{n-1} / (a_n b_{n-1} (zeta_{n-1} - zeta_n)
//                + zeta_{n-1} a_{n-1} (1 + ds a_n))
//   a^s = a zeta_{n+1}/zeta_n,  b^s = b (zeta_{n+1}/zeta_n)^2
// A shift freezes once |zeta| |r| <= tol |b| and its zeta is not updated
// further; the lowest shift carries the Krylov space and freezes last.

// batched |a_j|^2 and Re<a_j, b_j> + sigma |a_j|^2: member blockIdx.y, partial[j][block]
template <typename S>
__global__ void __launch_bounds__(BS) k_norm2_b(Field a, long stride, double *partial)
{
    a = member(a, blockIdx.y, stride);
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double t = 0;
    if (i < a.n) {
        cx<C> v[12];
        load_spinor<S, C>(a, i, v);
        for (int c = 0; c < 12; c++) t += double(v[c].re) * double(v[c].re) + double(v[c].im) * double(v[c].im);
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

template <typename S>
__global__ void __launch_bounds__(BS) k_redot_b(Field a, Field b, long stride, double sigma, double *partial)
{
    a = member(a, blockIdx.y, stride);
    b = member(b, blockIdx.y, stride);
    using C = Cof<S>;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double t = 0;
    if (i < a.n) {
        cx<C> u[12], v[12];
        load_spinor<S, C>(a, i, u);
        load_spinor<S, C>(b, i, v);
        for (int c = 0; c < 12; c++) {
            const double ur = double(u[c].re), ui = double(u[c].im);
            t += ur * (double(v[c].re) + sigma * ur) + ui * (double(v[c].im) + sigma * ui);
        }
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// out[j] = sum of nparts partials of member j (fixed order)
__global__ void __launch_bounds__(BS) k_finish_b(const double *partial, int nparts, double *out)
{
    double t = 0;
    for (int k = threadIdx.x; k < nparts; k += BS) t += partial[(long)blockIdx.x * nparts + k];
    t = block_sum(t);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Block Gram-Schmidt for flexible GCR.  FP64 or FP32 fields are viewed as flat
// complex arrays of m elements (the inner product does not depend on the
// layout); sums are accumulated in FP64.  A BF16 basis has its own kernels
// below.  Each thread owns GS_EPT elements of
// one chunk; partial sums are written per workgroup, member-major
// ([member][block]), and summed in a fixed order.

static constexpr int GS_EPT = 8;

static long gs_blocks(long m) { return (m + (long)BS * GS_EPT - 1) / ((long)BS * GS_EPT); }

template <typename T2>
__device__ __forceinline__ double2 ld2(const T2 *p, long k)
{
    const T2 v = p[k];
    return make_double2(double(v.x), double(v.y));
}

template <typename T2>
__device__ __forceinline__ void st2(T2 *p, long k, double2 v)
{
    using R = decltype(T2{}.x);
    p[k] = T2{R(v.x), R(v.y)};
}

// wave-level sum (no barrier); lane 0 holds the result
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// partial[(2j + {0,1}) nblk + blk] = Re, Im of sum conj(X_j) y over the chunk, j < nv.
// Each dot is reduced within the wavefront and the per-wave sums are kept in
// LDS; one barrier at the end instead of two per dot.
static constexpr int GS_MAXV = 64;
template <typename T2>
__global__ void __launch_bounds__(BS) k_gs_dots(const T2 *const *X, int nv, const T2 *y, long m, double *partial)
{
    __shared__ double red[2 * GS_MAXV][BS / 64];
    const long nblk = gridDim.x;
    const long base = (long)blockIdx.x * BS * GS_EPT + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 yv[GS_EPT];
#pragma unroll
    for (int e = 0; e < GS_EPT; e++) {
        const long k = base + (long)e * BS;
        yv[e] = k < m ? ld2(y, k) : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < nv; j++) {
        const T2 *x = X[j];
        double2 xv[GS_EPT];
#pragma unroll
        for (int e = 0; e < GS_EPT; e++) {
            const long k = base + (long)e * BS;
            xv[e] = k < m ? ld2(x, k) : make_double2(0.0, 0.0);
        }
        double re = 0, im = 0;
#pragma unroll
        for (int e = 0; e < GS_EPT; e++) {
            re += xv[e].x * yv[e].x + xv[e].y * yv[e].y;
            im += xv[e].x * yv[e].y - xv[e].y * yv[e].x;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            red[2 * j][wave] = re;
            red[2 * j + 1][wave] = im;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * nv; q += BS) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < BS / 64; w++) t += red[q][w];
        partial[(long)q * nblk + blockIdx.x] = t;
    }
}

// y -= sum_j b_j X_j, w -= sum_j b_j W_j with b_j = dots_j / nq[3 j] (dots_j =
// <X_j, y> as Re, Im pairs); partials of |y|^2 and <y, r> (new y) as members 0..2.
// The loop over j is outermost, so the loads of all elements of a thread for
// one j are in flight together.
template <typename T2>
__global__ void __launch_bounds__(BS) k_gs_project(const T2 *const *X, const T2 *const *W, int nv, const double *dots,
                                                   const double *nq, T2 *y, T2 *w, const T2 *r, long m,
                                                   double *partial)
{
    const long nblk = gridDim.x;
    const long base = (long)blockIdx.x * BS * GS_EPT + threadIdx.x;
    double2 yv[GS_EPT], wv[GS_EPT];
#pragma unroll
    for (int e = 0; e < GS_EPT; e++) {
        const long k = base + (long)e * BS;
        yv[e] = k < m ? ld2(y, k) : make_double2(0.0, 0.0);
        wv[e] = k < m ? ld2(w, k) : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < nv; j++) {
        const double inv = 1.0 / nq[3 * j];
        const double bre = dots[2 * j] * inv, bim = dots[2 * j + 1] * inv;
        const T2 *xj = X[j], *wj = W[j];
        T2 xr[GS_EPT], vr[GS_EPT];
#pragma unroll
        for (int e = 0; e < GS_EPT; e++) {
            const long k = base + (long)e * BS;
            if (k < m) {
                xr[e] = xj[k];
                vr[e] = wj[k];
            } else {
                xr[e] = T2{};
                vr[e] = T2{};
            }
        }
#pragma unroll
        for (int e = 0; e < GS_EPT; e++) {
            const double xx = double(xr[e].x), xy = double(xr[e].y), vx = double(vr[e].x), vy = double(vr[e].y);
            yv[e].x -= bre * xx - bim * xy;
            yv[e].y -= bre * xy + bim * xx;
            wv[e].x -= bre * vx - bim * vy;
            wv[e].y -= bre * vy + bim * vx;
        }
    }
    double n2 = 0, dre = 0, dim_ = 0;
#pragma unroll
    for (int e = 0; e < GS_EPT; e++) {
        const long k = base + (long)e * BS;
        if (k >= m) continue;
        st2(y, k, yv[e]);
        st2(w, k, wv[e]);
        const double2 ys = ld2(y, k);  // as stored
        const double2 rv = ld2(r, k);
        n2 += ys.x * ys.x + ys.y * ys.y;
        dre += ys.x * rv.x + ys.y * rv.y;
        dim_ += ys.x * rv.y - ys.y * rv.x;
    }
    n2 = block_sum(n2);
    dre = block_sum(dre);
    dim_ = block_sum(dim_);
    if (threadIdx.x == 0) {
        partial[0 * nblk + blockIdx.x] = n2;
        partial[1 * nblk + blockIdx.x] = dre;
        partial[2 * nblk + blockIdx.x] = dim_;
    }
}

// a = <q, r> / |q|^2 (coef = {|q|^2, Re, Im}); x += a z, r -= a q; partials |r|^2
template <typename T2>
__global__ void __launch_bounds__(BS) k_gs_update(T2 *x, const T2 *z, T2 *r, const T2 *q, const double *coef, long m,
                                                  double *partial)
{
    const long base = (long)blockIdx.x * BS * GS_EPT + threadIdx.x;
    const double inv = 1.0 / coef[0];
    const double are = coef[1] * inv, aim = coef[2] * inv;
    double n2 = 0;
#pragma unroll
    for (int e = 0; e < GS_EPT; e++) {
        const long k = base + (long)e * BS;
        if (k >= m) continue;
        const double2 zv = ld2(z, k), qv = ld2(q, k);
        double2 xv = ld2(x, k), rv = ld2(r, k);
        xv.x += are * zv.x - aim * zv.y;
        xv.y += are * zv.y + aim * zv.x;
        rv.x -= are * qv.x - aim * qv.y;
        rv.y -= are * qv.y + aim * qv.x;
        st2(x, k, xv);
        st2(r, k, rv);
        n2 += rv.x * rv.x + rv.y * rv.y;
    }
    n2 = block_sum(n2);
    if (threadIdx.x == 0) partial[blockIdx.x] = n2;
}

// The same three steps with the basis vectors stored in BF16 and the residual
// and solution in FP32.  A lane takes pairs of adjacent complex components:
// 8 bytes of a basis vector and the matching 16 bytes of the residual, GS_PPT
// pairs per lane, so that a lane keeps as many bytes in flight as the FP32
// kernels.  The projection is accumulated in FP32 (its result is rounded to
// BF16); sums are FP64.
//
// A field is stored as 16-byte planes, [plane][site][component in plane]:
// BF16 holds four complex components per plane, FP32 two.  Pair p of a BF16
// vector (components 4q + 2h and 4q + 2h + 1 of site i, p = 2 (q nsite + i) + h)
// is the 16-byte piece (2q + h) nsite + i of the FP32 field.
static constexpr int GS_PPT = 8;

static long gs_blocks_bf(long m) { return (m / 2 + (long)BS * GS_PPT - 1) / ((long)BS * GS_PPT); }

// a BF16 value is the upper half of the FP32 value; the lower 16 bits of a
// 32-bit word hold the real part, the upper the imaginary part
__device__ __forceinline__ float4 bf_pair(uint2 u)
{
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                       __uint_as_float(u.y & 0xffff0000u));
}

__device__ __forceinline__ unsigned bf_word(float re, float im)
{
    const __hip_bfloat162 t = __float22bfloat162_rn(make_float2(re, im));  // round to nearest even
    unsigned u;
    __builtin_memcpy(&u, &t, sizeof(u));
    return u;
}

__device__ __forceinline__ uint2 bf_pack(float4 v) { return make_uint2(bf_word(v.x, v.y), bf_word(v.z, v.w)); }

// the launchers check 12 nsite < 2^32, so the site arithmetic fits 32 bits
__device__ __forceinline__ long res_piece(long p, long nsite)
{
    const unsigned nu = (unsigned)nsite, quad = (unsigned)(p >> 1), h = (unsigned)(p & 1);
    const unsigned q = quad / nu, i = quad - q * nu;
    return (long)(2u * q + h) * nsite + i;
}

__global__ void __launch_bounds__(BS) k_gs_dots_bf(const uint2 *const *X, int nv, const uint2 *y, long m2,
                                                   double *partial)
{
    __shared__ double red[2 * GS_MAXV][BS / 64];
    const long nblk = gridDim.x;
    const long base = (long)blockIdx.x * BS * GS_PPT + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float4 yv[GS_PPT];
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) {
        const long k = base + (long)e * BS;
        yv[e] = k < m2 ? bf_pair(y[k]) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int j = 0; j < nv; j++) {
        const uint2 *x = X[j];
        uint2 xr[GS_PPT];
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const long k = base + (long)e * BS;
            xr[e] = k < m2 ? x[k] : make_uint2(0u, 0u);
        }
        double re = 0, im = 0;
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const float4 xv = bf_pair(xr[e]);
            re += double(xv.x) * yv[e].x + double(xv.y) * yv[e].y + double(xv.z) * yv[e].z + double(xv.w) * yv[e].w;
            im += double(xv.x) * yv[e].y - double(xv.y) * yv[e].x + double(xv.z) * yv[e].w - double(xv.w) * yv[e].z;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            red[2 * j][wave] = re;
            red[2 * j + 1][wave] = im;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * nv; q += BS) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < BS / 64; w++) t += red[q][w];
        partial[(long)q * nblk + blockIdx.x] = t;
    }
}

// PW false: only y is projected (w and W unused); the caller keeps its
// preconditioned directions as they were made and combines them at the restart
// with coefficients transformed by k_gs_raw_coef.
template <bool PW>
__global__ void __launch_bounds__(BS) k_gs_project_bf(const uint2 *const *X, const uint2 *const *W, int nv,
                                                      const double *dots, const double *nq, uint2 *y, uint2 *w,
                                                      const float4 *r, long m2, long nsite, double *partial)
{
    const long nblk = gridDim.x;
    const long base = (long)blockIdx.x * BS * GS_PPT + threadIdx.x;
    float4 yv[GS_PPT], wv[GS_PPT];
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) {
        const long k = base + (long)e * BS;
        yv[e] = k < m2 ? bf_pair(y[k]) : make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (PW) wv[e] = k < m2 ? bf_pair(w[k]) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int j = 0; j < nv; j++) {
        const double inv = 1.0 / nq[3 * j];
        const float bre = float(dots[2 * j] * inv), bim = float(dots[2 * j + 1] * inv);
        const uint2 *xj = X[j];
        uint2 xr[GS_PPT], vr[GS_PPT];
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const long k = base + (long)e * BS;
            xr[e] = k < m2 ? xj[k] : make_uint2(0u, 0u);
            if constexpr (PW) vr[e] = k < m2 ? W[j][k] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const float4 xd = bf_pair(xr[e]);
            yv[e].x -= bre * xd.x - bim * xd.y;
            yv[e].y -= bre * xd.y + bim * xd.x;
            yv[e].z -= bre * xd.z - bim * xd.w;
            yv[e].w -= bre * xd.w + bim * xd.z;
            if constexpr (PW) {
                const float4 vd = bf_pair(vr[e]);
                wv[e].x -= bre * vd.x - bim * vd.y;
                wv[e].y -= bre * vd.y + bim * vd.x;
                wv[e].z -= bre * vd.z - bim * vd.w;
                wv[e].w -= bre * vd.w + bim * vd.z;
            }
        }
    }
    double n2 = 0, dre = 0, dim_ = 0;
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) {
        const long k = base + (long)e * BS;
        if (k >= m2) continue;
        const uint2 yb = bf_pack(yv[e]);
        y[k] = yb;
        if constexpr (PW) w[k] = bf_pack(wv[e]);
        const float4 ys = bf_pair(yb);  // as stored
        const float4 rv = r[res_piece(k, nsite)];
        n2 += double(ys.x) * ys.x + double(ys.y) * ys.y + double(ys.z) * ys.z + double(ys.w) * ys.w;
        dre += double(ys.x) * rv.x + double(ys.y) * rv.y + double(ys.z) * rv.z + double(ys.w) * rv.w;
        dim_ += double(ys.x) * rv.y - double(ys.y) * rv.x + double(ys.z) * rv.w - double(ys.w) * rv.z;
    }
    n2 = block_sum(n2);
    dre = block_sum(dre);
    dim_ = block_sum(dim_);
    if (threadIdx.x == 0) {
        partial[0 * nblk + blockIdx.x] = n2;
        partial[1 * nblk + blockIdx.x] = dre;
        partial[2 * nblk + blockIdx.x] = dim_;
    }
}

// x += a z (skipped when x is null: the caller combines the cycle's directions
// into x at the restart, k_gs_combine_bf), r -= a q, partials of |r|^2; rb,
// if not null, receives the new r rounded to BF16 (in the basis layout)
__global__ void __launch_bounds__(BS) k_gs_update_bf(float4 *x, const uint2 *z, float4 *r, const uint2 *q,
                                                     const double *coef, long m2, long nsite, double *partial,
                                                     uint2 *rb)
{
    const long base = (long)blockIdx.x * BS * GS_PPT + threadIdx.x;
    const double inv = 1.0 / coef[0];
    const double are = coef[1] * inv, aim = coef[2] * inv;
    double n2 = 0;
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) {
        const long k = base + (long)e * BS;
        if (k >= m2) continue;
        const float4 qv = bf_pair(q[k]);
        const long kr = res_piece(k, nsite);
        if (x) {
            const float4 zv = bf_pair(z[k]);
            float4 xv = x[kr];
            xv.x = float(xv.x + (are * zv.x - aim * zv.y));
            xv.y = float(xv.y + (are * zv.y + aim * zv.x));
            xv.z = float(xv.z + (are * zv.z - aim * zv.w));
            xv.w = float(xv.w + (are * zv.w + aim * zv.z));
            x[kr] = xv;
        }
        float4 rv = r[kr];
        rv.x = float(rv.x - (are * qv.x - aim * qv.y));
        rv.y = float(rv.y - (are * qv.y + aim * qv.x));
        rv.z = float(rv.z - (are * qv.z - aim * qv.w));
        rv.w = float(rv.w - (are * qv.w + aim * qv.z));
        r[kr] = rv;
        if (rb) rb[k] = bf_pack(rv);
        n2 += double(rv.x) * rv.x + double(rv.y) * rv.y + double(rv.z) * rv.z + double(rv.w) * rv.w;
    }
    n2 = block_sum(n2);
    if (threadIdx.x == 0) partial[blockIdx.x] = n2;
}

// x += sum_j a_j Z_j over nz BF16 directions, oldest first, with a_j =
// (coef[3j+1] + i coef[3j+2]) / coef[3j]; x FP32
__global__ void __launch_bounds__(BS) k_gs_combine_bf(float4 *x, const uint2 *const *Z, int nz, const double *coef,
                                                      long m2, long nsite)
{
    const long base = (long)blockIdx.x * BS * GS_PPT + threadIdx.x;
    double4 acc[GS_PPT];
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) acc[e] = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int j = 0; j < nz; j++) {
        const double inv = 1.0 / coef[3 * j];
        const double are = coef[3 * j + 1] * inv, aim = coef[3 * j + 2] * inv;
        const uint2 *zj = Z[j];
        uint2 zr[GS_PPT];
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const long k = base + (long)e * BS;
            zr[e] = k < m2 ? zj[k] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int e = 0; e < GS_PPT; e++) {
            const float4 zv = bf_pair(zr[e]);
            acc[e].x += are * zv.x - aim * zv.y;
            acc[e].y += are * zv.y + aim * zv.x;
            acc[e].z += are * zv.z - aim * zv.w;
            acc[e].w += are * zv.w + aim * zv.z;
        }
    }
#pragma unroll
    for (int e = 0; e < GS_PPT; e++) {
        const long k = base + (long)e * BS;
        if (k >= m2) continue;
        const long kr = res_piece(k, nsite);
        float4 xv = x[kr];
        xv.x = float(xv.x + acc[e].x);
        xv.y = float(xv.y + acc[e].y);
        xv.z = float(xv.z + acc[e].z);
        xv.w = float(xv.w + acc[e].w);
        x[kr] = xv;
    }
}

// Solution coefficients for directions kept as they were made.  With the
// projected directions zt_k = z_k - sum_{j<k} b_jk zt_j (b_jk the projection
// coefficient of step k against vector j: dots[k stride + 2 j] / nq[3 j]),
// Z = Zt (1 + B) with B strictly upper triangular, so the update
// x += sum_k a_k zt_k (a_k = <q_k, r> / |q_k|^2 from nq) equals
// x += sum_k c_k z_k with (1 + B) c = a, solved by back substitution in FP64.
// cc[3k] = 1, cc[3k + 1 .. 2] = c_k, the form k_gs_combine_bf reads.  One thread.
__global__ void k_gs_raw_coef(int nz, int stride, const double *dots, const double *nq, double *cc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int k = nz - 1; k >= 0; k--) {
        const double inv = 1.0 / nq[3 * k];
        double re = nq[3 * k + 1] * inv, im = nq[3 * k + 2] * inv;
        for (int j = k + 1; j < nz; j++) {
            const double bre = dots[(long)j * stride + 2 * k] * inv, bim = dots[(long)j * stride + 2 * k + 1] * inv;
            const double cre = cc[3 * j + 1], cim = cc[3 * j + 2];
            re -= bre * cre - bim * cim;
            im -= bre * cim + bim * cre;
        }
        cc[3 * k] = 1.0;
        cc[3 * k + 1] = re;
        cc[3 * k + 2] = im;
    }
}

// r_j -= alpha_j (ap_j + sigma p_j) with alpha_j from the device, partial |r_j|^2
template <typename S>
__global__ void __launch_bounds__(BS) k_ms_residual(Field r, Field ap, Field p, double sigma, long stride,
                                                     const double *alpha, double *partial)
{
    r = member(r, blockIdx.y, stride);
    ap = member(ap, blockIdx.y, stride);
    p = member(p, blockIdx.y, stride);
    using C = Cof<S>;
    const C al = C(alpha[blockIdx.y]);
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    double t = 0;
    if (i < r.n) {
        cx<C> u[12], v[12];
        load_spinor<S, C>(r, i, u);
        load_spinor<S, C>(ap, i, v);
        if (sigma != 0.0) {
            cx<C> w[12];
            load_spinor<S, C>(p, i, w);
            for (int c = 0; c < 12; c++) v[c] = v[c] + C(sigma) * w[c];
        }
        for (int c = 0; c < 12; c++) {
            u[c] = u[c] - al * v[c];
            t += double(u[c].re) * double(u[c].re) + double(u[c].im) * double(u[c].im);
        }
        store_spinor<S, C>(r, i, u);
    }
    t = block_sum(t);
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// alpha_j = rho_j / <p_j, A p_j>; zero once every shift of rhs j is frozen
__global__ void k_ms_alpha(MsState s, int nrhs, int nshift)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrhs) return;
    int on = 0;
    for (int k = 0; k < nshift; k++) on |= s.active[k * nrhs + j];
    s.alpha[j] = (on && s.pap[j] > 0) ? s.rho[j] / s.pap[j] : 0.0;
}

// one workgroup per rhs j, one lane per shift; rho_new[j] holds |r_j|^2 after the update
__global__ void k_ms_recur(MsState s, const double *rho_new, int nrhs, int nshift, int kmin, int it)
{
    const int j = blockIdx.x, k = threadIdx.x;
    __shared__ int nact;
    if (k == 0) nact = 0;
    __syncthreads();
    const double al = s.alpha[j], alo = s.alpha_old[j], bo = s.beta_old[j];
    const double rho = s.rho[j], rn = rho_new[j];
    const double beta = (rho > 0 && al != 0.0) ? rn / rho : 0.0;
    if (k < nshift) {
        const int q = k * nrhs + j;
        double *cf = s.coef + 4 * (long)q;
        if (s.active[q] && al != 0.0) {
            const double ds = s.shifts[k] - s.shifts[kmin];
            const double z = s.zeta[q], zo = s.zeta_old[q];
            const double zn = z * zo * alo / (al * bo * (zo - z) + zo * alo * (1.0 + ds * al));
            cf[0] = al * zn / z;
            cf[1] = zn;
            cf[2] = beta * (zn / z) * (zn / z);
            cf[3] = 1.0;
            s.zeta_old[q] = z;
            s.zeta[q] = zn;
            s.iters[q] = it;
            atomicAdd(&nact, 1);
        } else {
            cf[3] = 0.0;
        }
    }
    __syncthreads();
    if (k < nshift) {
        const int q = k * nrhs + j;
        // freeze converged shifts; the Krylov carrier kmin only when it is the last one
        if (s.active[q] && s.coef[4 * (long)q + 3] != 0.0 && (k != kmin || nact == 1) &&
            fabs(s.zeta[q]) * sqrt(rn) <= s.target[j])
            s.active[q] = 0;
        if (!(rn == rn)) s.active[q] = 0;  // non-finite residual: stop this rhs
    }
    __syncthreads();
    if (k == 0 && al != 0.0) {
        s.rho[j] = rn;
        s.alpha_old[j] = al;
        s.beta_old[j] = beta;
    }
}

// Shifted directions and solutions of every active (shift, rhs) member:
// pnew = z r + b p, written to the other direction set Pn.  The solution
// updates go in pairs: with flush = 0 the update x += a p of this iteration
// is left pending (p stays in P); with flush = 1 x += a' p' of the previous
// iteration (coefficients cprev, direction in Pn, read before pnew overwrites
// it) and then x += a p are applied in one pass over x.  A member frozen in
// this iteration still receives its pending update.  For the Krylov carrier
// (shift kmin) the kernel also writes ta = (b + c P5) pnew, the operator's
// first factor, so that the next operator application starts from it; the
// workgroup holds whole fifth-dimension columns (Ls x sb lanes, one 4D site
// per row) and exchanges the carrier's new direction through LDS.
template <typename S>
__global__ void __launch_bounds__(256) k_ms_update_b(int nrhs, int nshift, int kmin, Field X, Field P, Field Pn,
                                                     Field r, Field ta, long stride, const double *coef,
                                                     const double *cprev, int flush, long vh, int Ls, double bb,
                                                     double cc, double mf)
{
    using C = Cof<S>;
    const int j = blockIdx.y;
    const int s = threadIdx.x, l = threadIdx.y;
    const long cb = (long)blockIdx.x * blockDim.y + l;
    const bool valid = cb < vh;
    const long i = cb * Ls + s;
    extern __shared__ unsigned char smem[];
    cx<C> *lds = (cx<C> *)smem;
    r = member(r, j, stride);
    cx<C> rv[12];
    if (valid) load_spinor<S, C>(r, i, rv);
    for (int k = 0; k < nshift; k++) {
        const long q = k * nrhs + j;
        const double *cf = coef + 4 * q;
        // both flags depend on the member only: the branch is uniform
        const bool on = cf[3] != 0.0, pend = flush && cprev[4 * q + 3] != 0.0;
        if (!on && !pend) continue;
        const Field p = member(P, q, stride), pn = member(Pn, q, stride);
        cx<C> pv[12];
        if (valid) {
            if (on) load_spinor<S, C>(p, i, pv);
            if (flush) {
                const Field x = member(X, q, stride);
                cx<C> xv[12];
                load_spinor<S, C>(x, i, xv);
                if (pend) {
                    const C ap = C(cprev[4 * q]);
                    cx<C> qv[12];
                    load_spinor<S, C>(pn, i, qv);
                    for (int c = 0; c < 12; c++) xv[c] = xv[c] + ap * qv[c];
                }
                if (on) {
                    const C a = C(cf[0]);
                    for (int c = 0; c < 12; c++) xv[c] = xv[c] + a * pv[c];
                }
                store_spinor<S, C>(x, i, xv);
            }
            if (on) {
                const C z = C(cf[1]), b = C(cf[2]);
                for (int c = 0; c < 12; c++) pv[c] = z * rv[c] + b * pv[c];
                store_spinor<S, C>(pn, i, pv);
                storage_round<S, C>(pv);
            }
        }
        if (k == kmin && on) {
            for (int c = 0; c < 12; c++) lds[(l * Ls + s) * 12 + c] = valid ? pv[c] : mk(C(0), C(0));
            __syncthreads();
            if (valid) {
                const cx<C> *blk = lds + l * Ls * 12;
                cx<C> out[12];
                for (int c = 0; c < 12; c++)
                    out[c] = C(bb) * pv[c] + C(cc) * shift5<C>(blk, c, s, Ls, false, C(mf));
                store_spinor<S, C>(member(ta, j, stride), i, out);
            }
        }
    }
}

// x += a p for the members whose update of the last iteration is still pending
template <typename S>
__global__ void __launch_bounds__(BS) k_ms_flush_b(int nrhs, int nshift, Field X, Field P, long stride,
                                                    const double *coef)
{
    using C = Cof<S>;
    const int j = blockIdx.y;
    const long i = blockIdx.x * (long)BS + threadIdx.x;
    if (i >= X.n) return;
    for (int k = 0; k < nshift; k++) {
        const long q = k * nrhs + j;
        if (coef[4 * q + 3] == 0.0) continue;
        const C a = C(coef[4 * q]);
        const Field x = member(X, q, stride), p = member(P, q, stride);
        cx<C> xv[12], pv[12];
        load_spinor<S, C>(x, i, xv);
        load_spinor<S, C>(p, i, pv);
        for (int c = 0; c < 12; c++) xv[c] = xv[c] + a * pv[c];
        store_spinor<S, C>(x, i, xv);
    }
}

void ms_launch_norm2(Context &c, int prec, Field a, int nb, long stride, double *out)
{
    const long np = (a.n + BS - 1) / BS;
    if (np * nb > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
    Timer tm(c, DWF_K_BLAS, nb * (12.0 * elem_bytes(prec)) * a.n, 0);
    DWF_DISPATCH(prec, k_norm2_b, dim3((unsigned)np, nb), dim3(BS), 0, a, stride, c.partials);
    hipLaunchKernelGGL(k_finish_b, dim3(nb), dim3(BS), 0, c.stream, c.partials, (int)np, out);
    HIPCHECK(hipGetLastError());
}

void ms_launch_redot(Context &c, int prec, Field a, Field b, int nb, long stride, double *out, double sigma)
{
    const long np = (a.n + BS - 1) / BS;
    if (np * nb > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
    Timer tm(c, DWF_K_BLAS, nb * 2 * (12.0 * elem_bytes(prec)) * a.n, 0);
    DWF_DISPATCH(prec, k_redot_b, dim3((unsigned)np, nb), dim3(BS), 0, a, b, stride, sigma, c.partials);
    hipLaunchKernelGGL(k_finish_b, dim3(nb), dim3(BS), 0, c.stream, c.partials, (int)np, out);
    HIPCHECK(hipGetLastError());
}

void ms_launch_step(Context &c, int prec, const MsState &s, Field r, Field ap, Field X, Field P, Field Pn,
                    const double *cprev, int nrhs, int nshift, int kmin, long stride, double *rho_new, int it,
                    Field pbase, double sigma, Field ta)
{
    const long np = (r.n + BS - 1) / BS;
    if (np * nrhs > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
    if (r.n != c.n5h) fail(DWF_EINVAL, "multi-shift fields must be half fields of the context");
    hipLaunchKernelGGL(k_ms_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, c.stream, s, nrhs, nshift);
    {
        Timer tm(c, DWF_K_BLAS, nrhs * (sigma != 0.0 ? 4 : 3) * (12.0 * elem_bytes(prec)) * r.n, 0);
        DWF_DISPATCH(prec, k_ms_residual, dim3((unsigned)np, nrhs), dim3(BS), 0, r, ap, pbase, sigma, stride, s.alpha,
                     c.partials);
    }
    hipLaunchKernelGGL(k_finish_b, dim3(nrhs), dim3(BS), 0, c.stream, c.partials, (int)np, rho_new);
    hipLaunchKernelGGL(k_ms_recur, dim3(nrhs), dim3(64), 0, c.stream, s, rho_new, nrhs, nshift, kmin, it);
    HIPCHECK(hipGetLastError());
    // pairs of iterations: the first (odd it) leaves its solution update pending
    const int flush = (it % 2 == 0) ? 1 : 0;
    const int Ls = c.Ls, sb = default_sb(c);
    const long nblk = (c.vh + sb - 1) / sb;
    const size_t lds = (size_t)sb * Ls * 12 * (prec == P_F64 ? 16 : 8);
    Timer tm(c, DWF_K_BLAS, nrhs * (2 + (flush ? 5.0 : 2.0) * nshift) * (12.0 * elem_bytes(prec)) * r.n, 0);
    DWF_DISPATCH(prec, k_ms_update_b, dim3((unsigned)nblk, nrhs), dim3(Ls, sb), lds, nrhs, nshift, kmin, X, P, Pn, r,
                 ta, stride, s.coef, cprev, flush, c.vh, Ls, c.p.b, c.p.c, c.p.mf);
}

void ms_launch_flush(Context &c, int prec, Field X, Field P, const double *coef, int nrhs, int nshift, long stride)
{
    const long np = (X.n + BS - 1) / BS;
    Timer tm(c, DWF_K_BLAS, nrhs * 3.0 * nshift * (12.0 * elem_bytes(prec)) * X.n, 0);
    DWF_DISPATCH(prec, k_ms_flush_b, dim3((unsigned)np, nrhs), dim3(BS), 0, nrhs, nshift, X, P, stride, coef);
}

// s-local operator of the form e0 + e1 P5 (dag: e0 + e1 P5^+): A, A^+, Mooee
// and Mooee^+, from the fifth-dimension neighbours alone instead of a dense
// Ls x Ls product (workgroup = Ls x sb lanes, one 4D site per row).  The
// Ls x 12 block of a 4D site is staged component-major in LDS, so consecutive
// lanes s touch consecutive words.  in and out may alias: every lane reads its
// own element before the barrier.
template <typename S>
__global__ void __launch_bounds__(256) k_slocal_shift(Field in, Field out, double e0, double e1, int dag, double mf,
                                                      long vh, int Ls, long bstride)
{
    using C = Cof<S>;
    in = member(in, blockIdx.y, bstride);
    out = member(out, blockIdx.y, bstride);
    const int s = threadIdx.x, j = threadIdx.y, sb = blockDim.y;
    const long cb = (long)blockIdx.x * sb + j;
    const bool valid = cb < vh;
    const long i = cb * Ls + s;
    extern __shared__ unsigned char smem[];
    cx<C> *rows = (cx<C> *)smem + (long)j * 12 * Ls;
    cx<C> v[12];
    if (valid) {
        load_spinor<S, C>(in, i, v);
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = mk(C(0), C(0));
    }
#pragma unroll
    for (int c = 0; c < 12; c++) rows[c * Ls + s] = v[c];
    __syncthreads();
    if (!valid) return;
    const C a0 = C(e0), a1 = C(e1);
    cx<C> res[12];
#pragma unroll
    for (int c = 0; c < 12; c++) res[c] = a0 * v[c] + a1 * shift5t<C>(rows, c, s, Ls, dag != 0, C(mf));
    store_spinor<S, C>(out, i, res);
}

void launch_slocal_shift(Context &c, int prec, double e0, double e1, bool dag, Field in, Field out, int nbatch,
                         long bstride)
{
    const int Ls = c.Ls, sb = default_sb(c);
    const long nblk = (c.vh + sb - 1) / sb;
    const int nb = std::max(1, nbatch);
    const size_t lds = (size_t)sb * Ls * 12 * (prec == P_F64 ? 16 : 8);
    const double fb = 12.0 * elem_bytes(prec) + (prec == P_F16 ? 4.0 : 0.0);
    Timer tm(c, DWF_K_SLOCAL, nb * 2.0 * fb * c.n5h, nb * 96.0 * c.n5h, prec);
    DWF_DISPATCH(prec, k_slocal_shift, dim3((unsigned)nblk, (unsigned)nb), dim3(Ls, sb), lds, in, out, e0, e1,
                 dag ? 1 : 0, c.p.mf, c.vh, Ls, nb > 1 ? bstride : 0L);
}

// plain 16-byte streaming copy, grid-stride
__global__ void __launch_bounds__(BS) k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, long n)
{
    for (long i = blockIdx.x * (long)BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) dst[i] = src[i];
}

// Bandwidth probes, the achievable-HBM references for the stencil's rooflines.
// Each lane keeps U independent 16-byte loads in flight per round (addresses
// a grid apart, so a round of the grid reads U contiguous blocks), loads and
// stores non-temporal when NT.  KIND 0: dst = a (copy); 1: read a only, each
// workgroup writes the XOR of what it read to dst[blockIdx.x]; 2: dst = a ^ b
// (two streams read per stream written, the hop's read:write mix).
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4u_t probe_load(const v4u_t *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT>
__device__ __forceinline__ void probe_store(v4u_t *p, v4u_t v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int KIND, int U, bool NT>
__global__ void __launch_bounds__(BS) k_stream_probe(const v4u_t *__restrict__ a, const v4u_t *__restrict__ b,
                                                     v4u_t *__restrict__ dst, long n)
{
    const long G = (long)gridDim.x * BS;
    const long t = blockIdx.x * (long)BS + threadIdx.x;
    v4u_t acc = {0u, 0u, 0u, 0u};
    for (long i0 = t; i0 < n; i0 += U * G) {
        v4u_t va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long i = i0 + u * G;
            if (i < n) {
                va[u] = probe_load<NT>(a + i);
                if constexpr (KIND == 2) vb[u] = probe_load<NT>(b + i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long i = i0 + u * G;
            if (i < n) {
                if constexpr (KIND == 0) probe_store<NT>(dst + i, va[u]);
                else if constexpr (KIND == 2) probe_store<NT>(dst + i, va[u] ^ vb[u]);
                else acc ^= va[u];
            }
        }
    }
    if constexpr (KIND == 1) {
        __shared__ v4u_t red[BS];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = BS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] ^= red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) dst[blockIdx.x] = red[0];
    }
}

long stream_probe_blocks(size_t bytes, int unroll)
{
    const long n = (long)(bytes / 16);
    return std::max<long>(1, std::min<long>((n + (long)BS * unroll - 1) / ((long)BS * unroll), 65536L));
}

void launch_stream_probe(Context &c, int kind, int unroll, bool nt, const void *a, const void *b, void *dst,
                         size_t bytes)
{
    const long n = (long)(bytes / 16);
    const long nblk = stream_probe_blocks(bytes, unroll);
    const double moved = kind == 0 ? 2.0 * bytes : (kind == 1 ? (double)bytes : 3.0 * bytes);
    Timer tm(c, DWF_K_BLAS, moved, 0);
    const v4u_t *pa = (const v4u_t *)a, *pb = (const v4u_t *)b;
    v4u_t *pd = (v4u_t *)dst;
#define DWF_PROBE(K, U)                                                                                        \
    do {                                                                                                       \
        if (nt)                                                                                                \
            hipLaunchKernelGGL((k_stream_probe<K, U, true>), dim3((unsigned)nblk), dim3(BS), 0, c.stream, pa, pb, \
                               pd, n);                                                                         \
        else                                                                                                   \
            hipLaunchKernelGGL((k_stream_probe<K, U, false>), dim3((unsigned)nblk), dim3(BS), 0, c.stream, pa,   \
                               pb, pd, n);                                                                     \
    } while (0)
#define DWF_PROBE_U(K)                        \
    do {                                      \
        switch (unroll) {                     \
        case 1: DWF_PROBE(K, 1); break;       \
        case 2: DWF_PROBE(K, 2); break;       \
        case 4: DWF_PROBE(K, 4); break;       \
        default: DWF_PROBE(K, 8); break;      \
        }                                     \
    } while (0)
    switch (kind) {
    case 0: DWF_PROBE_U(0); break;
    case 1: DWF_PROBE_U(1); break;
    default: DWF_PROBE_U(2); break;
    }
#undef DWF_PROBE_U
#undef DWF_PROBE
    HIPCHECK(hipGetLastError());
}

void launch_stream_copy(Context &c, const void *src, void *dst, size_t bytes)
{
    const long n = (long)(bytes / 16);
    const long nblk = std::min<long>((n + BS - 1) / BS, 65536L);
    Timer tm(c, DWF_K_BLAS, 2.0 * bytes, 0);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)std::max<long>(nblk, 1)), dim3(BS), 0, c.stream,
                       (const uint4 *)src, (uint4 *)dst, n);
    HIPCHECK(hipGetLastError());
}

// ------------------------------------------------------------ launchers

static double sbytes(int prec) { return 12.0 * elem_bytes(prec) + (prec == P_F16 ? 4.0 : 0.0); }

static void need_partials(Context &c, long n, int width)
{
    if (n * width > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
}

int launch_norm2(Context &c, int prec, Field a)
{
    const long nb = (a.n + BS - 1) / BS;
    need_partials(c, nb, 1);
    Timer tm(c, DWF_K_BLAS, sbytes(prec) * a.n, 4.0 * 12 * a.n);
    DWF_DISPATCH(prec, k_norm2, g1(a.n), dim3(BS), 0, a, c.partials);
    return (int)nb;
}

int launch_dot(Context &c, int prec, Field a, Field b)
{
    const long nb = (a.n + BS - 1) / BS;
    need_partials(c, nb, 2);
    Timer tm(c, DWF_K_BLAS, 2 * sbytes(prec) * a.n, 8.0 * 12 * a.n);
    DWF_DISPATCH(prec, k_dot, g1(a.n), dim3(BS), 0, a, b, c.partials);
    return (int)nb;
}

void launch_finish(Context &c, int nparts, int width, int slot, double *mirror, int qslot, int nslot)
{
    if (qslot >= 0 && (width != 1 || nslot < 0)) fail(DWF_EINVAL, "quotient needs one sum and a numerator slot");
    Timer tm(c, DWF_K_BLAS, 8.0 * nparts * width, 0);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(FBS), 0, c.stream, c.partials, nparts, width, c.dscal, slot, mirror,
                       qslot, nslot);
    HIPCHECK(hipGetLastError());
}

void launch_scalar_div(Context &c, int out, int num, int den)
{
    hipLaunchKernelGGL(k_scalar_div, dim3(1), dim3(64), 0, c.stream, c.dscal, out, num, den);
    HIPCHECK(hipGetLastError());
}

void launch_set_scalar(Context &c, int slot, double v)
{
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, c.stream, c.dscal, slot, v);
    HIPCHECK(hipGetLastError());
}

void launch_cg_beta(Context &c, int beta, int rho, int rho_new)
{
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, c.stream, c.dscal, beta, rho, rho_new);
    HIPCHECK(hipGetLastError());
}

void launch_axpby(Context &c, int prec, double a, Field x, double b, Field y, Field z)
{
    Timer tm(c, DWF_K_BLAS, 3 * sbytes(prec) * x.n, 36.0 * x.n);
    DWF_DISPATCH(prec, k_axpby, g1(x.n), dim3(BS), 0, a, x, b, y, z);
}

void launch_axpbypcz(Context &c, int prec, double a, Field x, double b, Field y, double cc, Field w, Field z)
{
    Timer tm(c, DWF_K_BLAS, 4 * sbytes(prec) * x.n, 60.0 * x.n);
    DWF_DISPATCH(prec, k_axpbypcz, g1(x.n), dim3(BS), 0, a, x, b, y, cc, w, z);
}

void launch_caxpy(Context &c, int prec, double are, double aim, Field x, Field y)
{
    Timer tm(c, DWF_K_BLAS, 3 * sbytes(prec) * x.n, 96.0 * x.n);
    DWF_DISPATCH(prec, k_caxpy, g1(x.n), dim3(BS), 0, are, aim, x, y);
}

void launch_zero(Context &c, int prec, Field a)
{
    Timer tm(c, DWF_K_BLAS, sbytes(prec) * a.n, 0);
    DWF_DISPATCH(prec, k_zero, g1(a.n), dim3(BS), 0, a);
}

void launch_copy(Context &c, int prec, Field a, Field b)
{
    Timer tm(c, DWF_K_BLAS, 2 * sbytes(prec) * a.n, 0);
    DWF_DISPATCH(prec, k_copy, g1(a.n), dim3(BS), 0, a, b);
}

int launch_cg_update_xr(Context &c, int prec, Field x, Field r, Field p, Field ap, int ia)
{
    const long nb = (x.n + BS - 1) / BS;
    need_partials(c, nb, 1);
    const int xp = accum_prec(prec);
    Timer tm(c, DWF_K_BLAS, (4 * sbytes(prec) + 2 * sbytes(xp)) * x.n, 120.0 * x.n);
    const dim3 grid = g1(x.n), blk(BS);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL((k_cg_update_xr<F64, F64>), grid, blk, 0, c.stream, x, r, p, ap, c.dscal, ia, c.partials); break;
    case P_F32: hipLaunchKernelGGL((k_cg_update_xr<F32, F32>), grid, blk, 0, c.stream, x, r, p, ap, c.dscal, ia, c.partials); break;
    case P_F16: hipLaunchKernelGGL((k_cg_update_xr<F16, F32>), grid, blk, 0, c.stream, x, r, p, ap, c.dscal, ia, c.partials); break;
    default: hipLaunchKernelGGL((k_cg_update_xr<BF16, F32>), grid, blk, 0, c.stream, x, r, p, ap, c.dscal, ia, c.partials); break;
    }
    HIPCHECK(hipGetLastError());
    return (int)nb;
}

// the low-precision vector kernels pair storage precision S with the
// accumulator precision of the solution (FP64 with FP64, FP32 otherwise)
#define DWF_DISPATCH_X(prec, KERNEL, grid, blk, lds, ...)                                                      \
    switch (prec) {                                                                                            \
    case P_F64: hipLaunchKernelGGL((KERNEL<F64, F64>), grid, blk, lds, c.stream, __VA_ARGS__); break;          \
    case P_F32: hipLaunchKernelGGL((KERNEL<F32, F32>), grid, blk, lds, c.stream, __VA_ARGS__); break;          \
    case P_F16: hipLaunchKernelGGL((KERNEL<F16, F32>), grid, blk, lds, c.stream, __VA_ARGS__); break;          \
    default: hipLaunchKernelGGL((KERNEL<BF16, F32>), grid, blk, lds, c.stream, __VA_ARGS__); break;            \
    }                                                                                                          \
    HIPCHECK(hipGetLastError())

void launch_cg_update_p(Context &c, int prec, Field r, Field p, Field pout, Field pa, int ib, Field x, int ia,
                        const CgOlder &older)
{
    const int Ls = c.Ls;
    const int sb = default_sb(c);
    const long nblk = (c.vh + sb - 1) / sb;
    const size_t csz = (prec == P_F64) ? 16 : 8;
    const size_t lds = (size_t)sb * Ls * 12 * csz;
    if (ia >= 0 && !x.data) fail(DWF_EINVAL, "solution update needs x");
    if (older.n < 0 || older.n > CgOlder::MAX || (older.n > 0 && ia < 0))
        fail(DWF_EINVAL, "older solution updates need x and at most three directions");
    for (int q = 0; q < older.n; q++)
        if (!older.dir[q].data || older.slot[q] < 0) fail(DWF_EINVAL, "older solution update without a direction");
    const double xb = ia >= 0 ? 2 * sbytes(accum_prec(prec)) + older.n * sbytes(prec) : 0.0;
    Timer tm(c, DWF_K_BLAS, (4 * sbytes(prec) + xb) * c.n5h, 96.0 * c.n5h, prec);
    DWF_DISPATCH_X(prec, k_cg_update_p, dim3((unsigned)nblk), dim3(Ls, sb), lds, r, p, pout, pa, x, older, c.dscal, ib,
                   ia, c.vh, Ls, c.p.b, c.p.c, c.p.mf);
}

void launch_axpy_dev(Context &c, int prec, Field x, Field p, int ia)
{
    Timer tm(c, DWF_K_BLAS, (sbytes(prec) + 2 * sbytes(accum_prec(prec))) * x.n, 48.0 * x.n, prec);
    DWF_DISPATCH_X(prec, k_axpy_dev, g1(x.n), dim3(BS), 0, x, p, c.dscal, ia);
}

int launch_residual(Context &c, Field b, Field ax, Field r)
{
    const long nb = (b.n + BS - 1) / BS;
    need_partials(c, nb, 1);
    Timer tm(c, DWF_K_BLAS, 3 * sbytes(P_F64) * b.n, 72.0 * b.n);
    hipLaunchKernelGGL(k_residual, g1(b.n), dim3(BS), 0, c.stream, b, ax, r, c.partials);
    HIPCHECK(hipGetLastError());
    return (int)nb;
}

void launch_accumulate_low(Context &c, int prec, Field xh, Field xl)
{
    Timer tm(c, DWF_K_BLAS, (3 * sbytes(P_F64) / 1.5 + 2 * sbytes(prec)) * xh.n, 24.0 * xh.n);
    DWF_DISPATCH(prec, k_accumulate_low, g1(xh.n), dim3(BS), 0, xh, xl);
}

long gs_partials_needed(const Context &c, int nv) { return gs_blocks(12 * c.n5h) * std::max(3, 2 * nv); }

// basis precision prec, residual and solution precision rprec: FP64/FP64,
// FP32/FP32 or BF16/FP32
static void gs_prec_check(int prec, int rprec, long m)
{
    const bool ok = (prec == P_F64 && rprec == P_F64) || (prec == P_F32 && rprec == P_F32) ||
                    (prec == P_BF16 && rprec == P_F32);
    if (!ok) fail(DWF_ENOTSUP, "Gram-Schmidt vectors must be FP64, FP32, or BF16 with an FP32 residual");
    if (m >= (1L << 32)) fail(DWF_ENOTSUP, "Gram-Schmidt vectors of 2^32 or more components");
}

static double gs_elem_bytes(int prec) { return prec == P_F64 ? 16.0 : prec == P_F32 ? 8.0 : 4.0; }

void launch_gs_dots(Context &c, int prec, const void *const *X_dev, int nv, Field y, double *partial, double *out)
{
    const long m = 12 * y.n, nblk = prec == P_BF16 ? gs_blocks_bf(m) : gs_blocks(m);
    gs_prec_check(prec, prec == P_BF16 ? P_F32 : prec, m);
    if (nv < 1 || nv > GS_MAXV) fail(DWF_EINVAL, "Gram-Schmidt block of 1..64 vectors");
    Timer tm(c, DWF_K_BLAS, (nv + 1.0) * gs_elem_bytes(prec) * m, 8.0 * nv * m, prec);
    if (prec == P_BF16)
        hipLaunchKernelGGL(k_gs_dots_bf, dim3((unsigned)nblk), dim3(BS), 0, c.stream, (const uint2 *const *)X_dev, nv,
                           (const uint2 *)y.data, m / 2, partial);
    else if (prec == P_F64)
        hipLaunchKernelGGL(k_gs_dots<double2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const double2 *const *)X_dev, nv, (const double2 *)y.data, m, partial);
    else
        hipLaunchKernelGGL(k_gs_dots<float2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const float2 *const *)X_dev, nv, (const float2 *)y.data, m, partial);
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(k_finish_b, dim3(2 * nv), dim3(BS), 0, c.stream, partial, (int)nblk, out);
    HIPCHECK(hipGetLastError());
}

void launch_gs_project(Context &c, int prec, int rprec, const void *const *X_dev, const void *const *W_dev, int nv,
                       const double *dots, const double *nq, Field y, Field w, Field r, double *partial, double *out)
{
    const long m = 12 * y.n, nblk = prec == P_BF16 ? gs_blocks_bf(m) : gs_blocks(m);
    gs_prec_check(prec, rprec, m);
    const bool pw = w.data != nullptr;
    if (!pw && (prec != P_BF16 || W_dev)) fail(DWF_EINVAL, "projection of y alone needs a BF16 basis and no W");
    const double vecs = pw ? 2.0 * nv + 4.0 : nv + 2.0;
    Timer tm(c, DWF_K_BLAS, (vecs * gs_elem_bytes(prec) + gs_elem_bytes(rprec)) * m,
             ((pw ? 16.0 : 8.0) * nv + 12.0) * m, prec);
    if (prec == P_BF16 && pw)
        hipLaunchKernelGGL(k_gs_project_bf<true>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const uint2 *const *)X_dev, (const uint2 *const *)W_dev, nv, dots, nq, (uint2 *)y.data,
                           (uint2 *)w.data, (const float4 *)r.data, m / 2, y.n, partial);
    else if (prec == P_BF16)
        hipLaunchKernelGGL(k_gs_project_bf<false>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const uint2 *const *)X_dev, (const uint2 *const *)nullptr, nv, dots, nq,
                           (uint2 *)y.data, (uint2 *)nullptr, (const float4 *)r.data, m / 2, y.n, partial);
    else if (prec == P_F64)
        hipLaunchKernelGGL(k_gs_project<double2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const double2 *const *)X_dev, (const double2 *const *)W_dev, nv, dots, nq,
                           (double2 *)y.data, (double2 *)w.data, (const double2 *)r.data, m, partial);
    else
        hipLaunchKernelGGL(k_gs_project<float2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream,
                           (const float2 *const *)X_dev, (const float2 *const *)W_dev, nv, dots, nq,
                           (float2 *)y.data, (float2 *)w.data, (const float2 *)r.data, m, partial);
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(k_finish_b, dim3(3), dim3(BS), 0, c.stream, partial, (int)nblk, out);
    HIPCHECK(hipGetLastError());
}

int launch_gs_update(Context &c, int prec, int rprec, Field x, Field z, Field r, Field q, const double *coef,
                     Field rb)
{
    const long m = 12 * r.n, nblk = prec == P_BF16 ? gs_blocks_bf(m) : gs_blocks(m);
    gs_prec_check(prec, rprec, m);
    if (!x.data && prec != P_BF16) fail(DWF_EINVAL, "Gram-Schmidt update needs x");
    need_partials(c, nblk, 1);
    if (rb.data && (prec != P_BF16 || rb.n != r.n)) fail(DWF_EINVAL, "BF16 residual copy needs a BF16 basis");
    const double xb = x.data ? gs_elem_bytes(prec) + 2.0 * gs_elem_bytes(rprec) : 0.0;
    const double rbb = rb.data ? gs_elem_bytes(P_BF16) : 0.0;
    Timer tm(c, DWF_K_BLAS, (gs_elem_bytes(prec) + 2.0 * gs_elem_bytes(rprec) + xb + rbb) * m, 18.0 * m, prec);
    if (prec == P_BF16)
        hipLaunchKernelGGL(k_gs_update_bf, dim3((unsigned)nblk), dim3(BS), 0, c.stream, (float4 *)x.data,
                           (const uint2 *)z.data, (float4 *)r.data, (const uint2 *)q.data, coef, m / 2, r.n,
                           c.partials, (uint2 *)rb.data);
    else if (prec == P_F64)
        hipLaunchKernelGGL(k_gs_update<double2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream, (double2 *)x.data,
                           (const double2 *)z.data, (double2 *)r.data, (const double2 *)q.data, coef, m, c.partials);
    else
        hipLaunchKernelGGL(k_gs_update<float2>, dim3((unsigned)nblk), dim3(BS), 0, c.stream, (float2 *)x.data,
                           (const float2 *)z.data, (float2 *)r.data, (const float2 *)q.data, coef, m, c.partials);
    HIPCHECK(hipGetLastError());
    return (int)nblk;
}

void launch_gs_combine(Context &c, int prec, Field x, const void *const *Z_dev, int nz, const double *coef)
{
    const long m = 12 * x.n, nblk = gs_blocks_bf(m);
    gs_prec_check(prec, P_F32, m);
    if (prec != P_BF16) fail(DWF_ENOTSUP, "deferred solution combination needs a BF16 basis");
    if (nz < 1 || nz > GS_MAXV) fail(DWF_EINVAL, "combination of 1..64 directions");
    Timer tm(c, DWF_K_BLAS, (nz * 4.0 + 16.0) * m, 8.0 * nz * m, prec);
    hipLaunchKernelGGL(k_gs_combine_bf, dim3((unsigned)nblk), dim3(BS), 0, c.stream, (float4 *)x.data,
                       (const uint2 *const *)Z_dev, nz, coef, m / 2, x.n);
    HIPCHECK(hipGetLastError());
}

void launch_gs_raw_coef(Context &c, int nz, int stride, const double *dots, const double *nq, double *cc)
{
    if (nz < 1 || nz > GS_MAXV || stride < 2 * nz) fail(DWF_EINVAL, "raw-direction coefficients of 1..64 directions");
    hipLaunchKernelGGL(k_gs_raw_coef, dim3(1), dim3(64), 0, c.stream, nz, stride, dots, nq, cc);
    HIPCHECK(hipGetLastError());
}

void launch_ms_update(Context &c, int prec, int nshift, Field *x, Field *p, Field r, const double *coef_dev,
                      const int *active_host)
{
    int nact = 0;
    for (int k = 0; k < nshift; k++) nact += active_host[k] ? 1 : 0;
    Timer tm(c, DWF_K_BLAS, (1 + 4.0 * nact) * sbytes(prec) * r.n, 96.0 * nact * r.n);
    DWF_DISPATCH(prec, k_ms_update, g1(r.n), dim3(BS), 0, nshift, (const Field *)x, (const Field *)p, r, coef_dev);
}

}  // namespace dwf
