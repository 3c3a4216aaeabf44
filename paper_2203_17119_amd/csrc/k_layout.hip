// Layout kernels: neighbour table, Dirichlet link preparation, and the
// conversions between the canonical FP64 layouts of the C ABI and the internal
// structure-of-arrays layouts in every storage precision.
#include <vector>

#include "dwf_internal.h"

namespace dwf {

struct Geo {
    int L[4];
    long vh;
    int Ls;
    const int *perm_inv;  // internal site j -> checkerboard index cb
};

// lexicographic site of checkerboard index cb in parity p (Lx is even, so
// sites 2cb and 2cb+1 differ only in x and exactly one has parity p)
__host__ __device__ __forceinline__ long site_of_cb(const int L[4], long cb, int p, int x[4])
{
    long n = 2 * cb, r = n;
    for (int mu = 0; mu < 4; mu++) {
        x[mu] = (int)(r % L[mu]);
        r /= L[mu];
    }
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != p) {
        n += 1;
        x[0] += 1;
    }
    return n;
}

__host__ __device__ __forceinline__ long lex(const int L[4], const int x[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

// Cache-blocked site order.  A workgroup's neighbours in +-x, +-y, +-z and
// +-t must still be in the L2 of its XCD when they are read again; in
// lexicographic order the +-t neighbours lie a whole 3D slice away.  Sites are
// therefore grouped in columns with a small (x/2, y, z) cross-section that run
// along t; a column's t-planes are consecutive, so a sweep along one column
// keeps about three planes live.  The order is a permutation of the
// checkerboard index cb = (x/2, y, z, t) and hence identical for both parities.
static long divisor_at_most(long n, long cap)
{
    for (long d = std::min(n, std::max(1L, cap)); d >= 1; d--)
        if (n % d == 0) return d;
    return 1;
}

void build_order(Context &c, int cxh, int cy, int cz)
{
    const int Lxh = c.L[0] / 2, Ly = c.L[1], Lz = c.L[2], Lt = c.L[3];
    if (cxh <= 0 || cy <= 0 || cz <= 0) {
        // target: one t-plane of a column about 0.6 MB in FP32 storage
        const long target = std::max(64L, 600000L / (96L * c.Ls));
        if ((long)Lxh * Ly * Lz <= 2 * target) {
            cxh = Lxh, cy = Ly, cz = Lz;
        } else {
            long best = -1;
            double best_face = 1e9;
            for (long dx = 1; dx <= Lxh; dx++) {
                if (Lxh % dx) continue;
                for (long dy = 1; dy <= Ly; dy++) {
                    if (Ly % dy) continue;
                    const long dz = divisor_at_most(Lz, target / (dx * dy));
                    const long plane = dx * dy * dz;
                    if (plane > target) continue;
                    // neighbour reads leaving the column per site
                    const double face = 1.0 / (2 * dx) + 1.0 / dy + 1.0 / dz;
                    if (plane > best || (plane == best && face < best_face)) {
                        best = plane;
                        best_face = face;
                        cxh = (int)dx, cy = (int)dy, cz = (int)dz;
                    }
                }
            }
        }
    }
    if (Lxh % cxh || Ly % cy || Lz % cz) fail(DWF_EINVAL, "column cross-section must divide (Lx/2, Ly, Lz)");
    c.order[0] = cxh, c.order[1] = cy, c.order[2] = cz;
    c.perm_h.assign(c.vh, 0);
    c.perm_inv_h.assign(c.vh, 0);
    long j = 0;
    for (int Z = 0; Z < Lz / cz; Z++)
        for (int Y = 0; Y < Ly / cy; Y++)
            for (int X = 0; X < Lxh / cxh; X++)
                for (int t = 0; t < Lt; t++)
                    for (int z = Z * cz; z < (Z + 1) * cz; z++)
                        for (int y = Y * cy; y < (Y + 1) * cy; y++)
                            for (int xh = X * cxh; xh < (X + 1) * cxh; xh++) {
                                const long cb = xh + (long)Lxh * (y + (long)Ly * (z + (long)Lz * t));
                                c.perm_h[cb] = (int)j;
                                c.perm_inv_h[j] = (int)cb;
                                j++;
                            }
    if (!c.perm_inv) HIPCHECK(hipMalloc(&c.perm_inv, c.vh * sizeof(int)));
    HIPCHECK(hipMemcpy(c.perm_inv, c.perm_inv_h.data(), c.vh * sizeof(int), hipMemcpyHostToDevice));
}

// sites in one column (one parity)
long column_sites(const Context &c) { return (long)c.order[0] * c.order[1] * c.order[2] * c.L[3]; }

// nbr[p][d][j]: internal index of the neighbour of site j (output parity p) in
// direction d, or -1 where the link crosses a Dirichlet face (it is zero, so
// the kernels skip the neighbour instead of reading across the block).  The
// stencil reads the same table site-major, nbr_sm[p][j][d]: the eight indices
// of the sites of one workgroup are then one contiguous block.
void build_neighbours(Context &c)
{
    std::vector<int> h((size_t)2 * 8 * c.vh), hs((size_t)2 * 8 * c.vh);
    for (int p = 0; p < 2; p++)
        for (long j = 0; j < c.vh; j++) {
            int x[4];
            site_of_cb(c.L, c.perm_inv_h[j], p, x);
            for (int d = 0; d < 8; d++) {
                const int mu = d & 3, step = d < 4 ? 1 : -1;
                const bool cut = c.p.dirichlet[mu] && (d < 4 ? x[mu] == c.L[mu] - 1 : x[mu] == 0);
                int y[4] = {x[0], x[1], x[2], x[3]};
                y[mu] = (y[mu] + step + c.L[mu]) % c.L[mu];
                const int nb = cut ? -1 : c.perm_h[lex(c.L, y) >> 1];
                h[((size_t)p * 8 + d) * c.vh + j] = nb;
                hs[((size_t)p * c.vh + j) * 8 + d] = nb;
            }
        }
    HIPCHECK(hipMemcpy(c.nbr, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(c.nbr_sm, hs.data(), hs.size() * sizeof(int), hipMemcpyHostToDevice));
}

// links of output parity p, entry k = 3 r + col of direction d at internal
// site j: U_mu(x) (d < 4) or U_mu(x-mu)^+ (d >= 4), zero when the link crosses
// a Dirichlet face (leaves through x_mu = L_mu - 1).  site_major: [j][d][k]
// (the 72 entries of a site contiguous, read by the stencil one workgroup
// block at a time); else [d][k][j] (read per lane by the network kernels).
template <typename S>
__global__ void k_prepare_links(Geo g, const double2 *gauge, int p, int4 dir, typename S::elem *out, int site_major)
{
    const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (j >= g.vh) return;
    int x[4];
    const long n = site_of_cb(g.L, g.perm_inv[j], p, x);
    const int dm[4] = {dir.x, dir.y, dir.z, dir.w};
    for (int d = 0; d < 8; d++) {
        const int mu = d & 3;
        long m = n;
        bool zero;
        if (d < 4) {
            zero = dm[mu] && x[mu] == g.L[mu] - 1;
        } else {
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = (y[mu] - 1 + g.L[mu]) % g.L[mu];
            m = lex(g.L, y);
            zero = dm[mu] && y[mu] == g.L[mu] - 1;
        }
        const double2 *U = gauge + (m * 4 + mu) * 9;
        for (int r = 0; r < 3; r++)
            for (int col = 0; col < 3; col++) {
                cx<double> v;
                if (d < 4) v = mk(U[r * 3 + col].x, U[r * 3 + col].y);
                else v = mk(U[col * 3 + r].x, -U[col * 3 + r].y);
                if (zero) v = mk(0.0, 0.0);
                const long k = (long)d * 9 + r * 3 + col;
                const long idx = site_major ? j * 72 + k : k * g.vh + j;
                if constexpr (LinkQ15<S>::value) ((uint32_t *)out)[idx] = pack_q15(v.re, v.im);
                else out[idx] = pack<S, double>(v);
            }
    }
}

static Geo geo(const Context &c)
{
    Geo g;
    for (int mu = 0; mu < 4; mu++) g.L[mu] = c.L[mu];
    g.vh = c.vh;
    g.perm_inv = c.perm_inv;
    g.Ls = c.Ls;
    return g;
}

void prepare_links(Context &c, int prec)
{
    const Geo g = geo(c);
    const int4 dir = make_int4(c.p.dirichlet[0], c.p.dirichlet[1], c.p.dirichlet[2], c.p.dirichlet[3]);
    const size_t bytes = (size_t)8 * 9 * c.vh * elem_bytes(prec);
    for (int p = 0; p < 2; p++) {
        if (!c.links[prec][p]) HIPCHECK(hipMalloc(&c.links[prec][p], bytes));
        const dim3 grid((unsigned)((c.vh + 255) / 256)), blk(256);
        const double2 *U = (const double2 *)c.gauge_canon;
        switch (prec) {
        case P_F64: hipLaunchKernelGGL(k_prepare_links<F64>, grid, blk, 0, c.stream, g, U, p, dir, (double2 *)c.links[prec][p], 1); break;
        case P_F32: hipLaunchKernelGGL(k_prepare_links<F32>, grid, blk, 0, c.stream, g, U, p, dir, (float2 *)c.links[prec][p], 1); break;
        case P_F16: hipLaunchKernelGGL(k_prepare_links<F16>, grid, blk, 0, c.stream, g, U, p, dir, (__half2 *)c.links[prec][p], 1); break;
        default: hipLaunchKernelGGL(k_prepare_links<BF16>, grid, blk, 0, c.stream, g, U, p, dir, (__hip_bfloat162 *)c.links[prec][p], 1); break;
        }
        HIPCHECK(hipGetLastError());
        if (prec == P_F32) {
            if (!c.links_net[p]) HIPCHECK(hipMalloc(&c.links_net[p], bytes));
            hipLaunchKernelGGL(k_prepare_links<F32>, grid, blk, 0, c.stream, g, U, p, dir, (float2 *)c.links_net[p], 0);
            HIPCHECK(hipGetLastError());
        }
    }
}

// canonical [n or cb][s][12] FP64 -> internal, one parity
template <typename S>
__global__ void k_import(Geo g, const double2 *canon, Field out, int full, int parity)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= g.vh * g.Ls) return;
    const long j = i / g.Ls;
    const int s = (int)(i - j * g.Ls);
    const long cb = g.perm_inv[j];
    long site = cb;
    if (full) {
        int x[4];
        site = site_of_cb(g.L, cb, parity, x);
    }
    const double2 *src = canon + (site * g.Ls + s) * 12;
    cx<double> v[12];
    for (int c = 0; c < 12; c++) v[c] = mk(src[c].x, src[c].y);
    store_spinor<S, double>(out, i, v);
}

template <typename S>
__global__ void k_export(Geo g, Field in, double2 *canon, int full, int parity)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= g.vh * g.Ls) return;
    const long j = i / g.Ls;
    const int s = (int)(i - j * g.Ls);
    const long cb = g.perm_inv[j];
    long site = cb;
    if (full) {
        int x[4];
        site = site_of_cb(g.L, cb, parity, x);
    }
    double2 *dst = canon + (site * g.Ls + s) * 12;
    cx<double> v[12];
    load_spinor<S, double>(in, i, v);
    for (int c = 0; c < 12; c++) dst[c] = make_double2(v[c].re, v[c].im);
}

template <typename SI, typename SO>
__global__ void k_convert(Field in, Field out)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= in.n) return;
    cx<double> v[12];
    load_spinor<SI, double>(in, i, v);
    store_spinor<SO, double>(out, i, v);
}

static dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

void launch_import(Context &c, int prec, const double *canon, Field out, int full, int parity)
{
    const Geo g = geo(c);
    const double2 *src = (const double2 *)canon;
    Timer tm(c, DWF_K_BLAS, (double)c.n5h * (192.0 + 12 * elem_bytes(prec)), 0);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_import<F64>, grid1(c.n5h), dim3(256), 0, c.stream, g, src, out, full, parity); break;
    case P_F32: hipLaunchKernelGGL(k_import<F32>, grid1(c.n5h), dim3(256), 0, c.stream, g, src, out, full, parity); break;
    case P_F16: hipLaunchKernelGGL(k_import<F16>, grid1(c.n5h), dim3(256), 0, c.stream, g, src, out, full, parity); break;
    default: hipLaunchKernelGGL(k_import<BF16>, grid1(c.n5h), dim3(256), 0, c.stream, g, src, out, full, parity); break;
    }
    HIPCHECK(hipGetLastError());
}

void launch_export(Context &c, int prec, Field in, double *canon, int full, int parity)
{
    const Geo g = geo(c);
    double2 *dst = (double2 *)canon;
    Timer tm(c, DWF_K_BLAS, (double)c.n5h * (192.0 + 12 * elem_bytes(prec)), 0);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_export<F64>, grid1(c.n5h), dim3(256), 0, c.stream, g, in, dst, full, parity); break;
    case P_F32: hipLaunchKernelGGL(k_export<F32>, grid1(c.n5h), dim3(256), 0, c.stream, g, in, dst, full, parity); break;
    case P_F16: hipLaunchKernelGGL(k_export<F16>, grid1(c.n5h), dim3(256), 0, c.stream, g, in, dst, full, parity); break;
    default: hipLaunchKernelGGL(k_export<BF16>, grid1(c.n5h), dim3(256), 0, c.stream, g, in, dst, full, parity); break;
    }
    HIPCHECK(hipGetLastError());
}

template <typename SI>
static void convert_to(Context &c, int pout, Field in, Field out)
{
    switch (pout) {
    case P_F64: hipLaunchKernelGGL((k_convert<SI, F64>), grid1(in.n), dim3(256), 0, c.stream, in, out); break;
    case P_F32: hipLaunchKernelGGL((k_convert<SI, F32>), grid1(in.n), dim3(256), 0, c.stream, in, out); break;
    case P_F16: hipLaunchKernelGGL((k_convert<SI, F16>), grid1(in.n), dim3(256), 0, c.stream, in, out); break;
    default: hipLaunchKernelGGL((k_convert<SI, BF16>), grid1(in.n), dim3(256), 0, c.stream, in, out); break;
    }
}

void launch_convert(Context &c, int pin, Field in, int pout, Field out)
{
    Timer tm(c, DWF_K_BLAS, (double)in.n * 12 * (elem_bytes(pin) + elem_bytes(pout)), 0);
    switch (pin) {
    case P_F64: convert_to<F64>(c, pout, in, out); break;
    case P_F32: convert_to<F32>(c, pout, in, out); break;
    case P_F16: convert_to<F16>(c, pout, in, out); break;
    default: convert_to<BF16>(c, pout, in, out); break;
    }
    HIPCHECK(hipGetLastError());
}

// ----------------------------------------------------------- domain boundary
//
// The two-flavour boundary action splits the lattice into a domain Omega and
// its complement (Sec. 2.1); mask[n] over the lexicographic 4D sites is
// nonzero on Omega.  The boundary is found by comparing the mask with its
// shift by one site in each direction (Sec. 2.4, "Results").

__host__ __device__ __forceinline__ long shifted(const int L[4], const int x[4], int mu, int step)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + step + L[mu]) % L[mu];
    return lex(L, y);
}

// U_mu(x) = 0 where x and x + mu lie in different domains; canonical FP64
// gauge [n][mu][3][3], one thread per (n, mu)
__global__ void k_mask_links(Geo g, const int8_t *mask, const double2 *gin, double2 *gout)
{
    const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long V = 2 * g.vh;
    if (k >= 4 * V) return;
    const long n = k / 4;
    const int mu = (int)(k - 4 * n);
    long r = n;
    int x[4];
    for (int d = 0; d < 4; d++) {
        x[d] = (int)(r % g.L[d]);
        r /= g.L[d];
    }
    const bool cut = (mask[n] != 0) != (mask[shifted(g.L, x, mu, 1)] != 0);
    for (int e = 0; e < 9; e++) gout[k * 9 + e] = cut ? make_double2(0.0, 0.0) : gin[k * 9 + e];
}

// gamma_mu psi_a = f_a psi_perm(a) per colour in the chiral basis
// gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_t = [[0, 1], [1, 0]]
__device__ __forceinline__ cx<double> gamma_row(int mu, int a, const cx<double> v[12], int col)
{
    const int src = mu < 2 ? 3 - a : (a ^ 2);
    const cx<double> u = v[src * 3 + col];
    switch (mu) {
    case 0: return (a < 2) ? mk(u.im, -u.re) : mk(-u.im, u.re);               // -i, -i, i, i
    case 1: return (a == 0 || a == 3) ? mk(-u.re, -u.im) : u;                 // -1, 1, 1, -1
    case 2: return (a == 0 || a == 3) ? mk(u.im, -u.re) : mk(-u.im, u.re);    // -i, i, i, -i
    default: return u;                                                         // 1, 1, 1, 1
    }
}

// kind 0: the spin-space mask of the boundary sites of Omega: (1 + gamma_mu)/2
// at a site whose only neighbour outside Omega is x + mu, (1 - gamma_mu)/2 if
// it is x - mu, 1 with two or more, 0 at every other site; kind 1: the field
// on Omega, zero outside.  One parity of an FP64 internal field.
__global__ void k_boundary_mask(Geo g, const int8_t *mask, Field in, Field out, int parity, int kind)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= g.vh * g.Ls) return;
    const long j = i / g.Ls;
    int x[4];
    const long n = site_of_cb(g.L, g.perm_inv[j], parity, x);
    cx<double> v[12];
    load_spinor<F64, double>(in, i, v);
    const bool inside = mask[n] != 0;
    int nout = 0, mu0 = 0, sg0 = 1;
    if (inside && kind == 0)
        for (int mu = 0; mu < 4; mu++)
            for (int sg = 1; sg >= -1; sg -= 2)
                if (mask[shifted(g.L, x, mu, sg)] == 0) {
                    nout++;
                    mu0 = mu;
                    sg0 = sg;
                }
    if (!inside || (kind == 0 && nout == 0)) {
        for (int c = 0; c < 12; c++) v[c] = mk(0.0, 0.0);
    } else if (kind == 0 && nout == 1) {
        cx<double> w[12];
        for (int a = 0; a < 4; a++)
            for (int col = 0; col < 3; col++) {
                const cx<double> gv = gamma_row(mu0, a, v, col);
                w[a * 3 + col] = 0.5 * (v[a * 3 + col] + double(sg0) * gv);
            }
        for (int c = 0; c < 12; c++) v[c] = w[c];
    }
    store_spinor<F64, double>(out, i, v);
}

void launch_mask_links(Context &c, const int8_t *mask, const double *gin, double *gout)
{
    const Geo g = geo(c);
    hipLaunchKernelGGL(k_mask_links, grid1(8 * c.vh), dim3(256), 0, c.stream, g, mask, (const double2 *)gin,
                       (double2 *)gout);
    HIPCHECK(hipGetLastError());
}

void launch_boundary_mask(Context &c, const int8_t *mask, Field in, Field out, int parity, int kind)
{
    const Geo g = geo(c);
    hipLaunchKernelGGL(k_boundary_mask, grid1(c.n5h), dim3(256), 0, c.stream, g, mask, in, out, parity, kind);
    HIPCHECK(hipGetLastError());
}

}  // namespace dwf
