// Fused domain-wall stencil for gfx950, included once per storage precision.
//
//   out(x,s) = sigma * Self(self)(x,s) + tau * Epi( H_{p,1-p} in )(x,s)
//
// H is the Wilson hop on every fifth-dimension slice: eight directions, the
// neighbour spinor projected to a half spinor (two colour vectors) with the
// chiral-basis identities
//   (1 + P g_k) psi = (h, P i sigma_k h),  h = u - P i sigma_k l   (k = x,y,z)
//   (1 + P g_t) psi = (h, P h),            h = u + P l
// (u, l = upper and lower spin pairs), the two colour vectors multiplied by the
// link and the lower pair rebuilt from the upper one.  P = -1 for the forward
// and +1 for the backward hop, both flipped for H^+ = g5 H g5.
//
// Work mapping: a workgroup is an (Ls x sb) grid of lanes, lane (s, j) owns the
// 5D site (cb, s) of 4D site cb = tile*sb + j.  The Ls lanes of one 4D site
// load the same link addresses, so each link is fetched from memory once per
// workgroup and reused for every s.  Fifth-dimension operators (Epi, Self)
// need every s of a site and run from LDS after one barrier:
//   Epi  = dense Ls x Ls matrix per chirality, or e0 + e1 P5 (P5^+), or a
//          Toeplitz operator (see below)
//   Self = s0 + s1 P5 (P5^+) on a second input at the output site.
//
// Toeplitz epilogue.  A A Mee^-1-type operator is, on each chirality, a
// polynomial in the twisted shift S (row s takes s-1, S^Ls = -mf): with first
// column f_k it is  T[t][s'] = f_{t-s'} (t >= s'),  -mf f_{t-s'+Ls} (t < s'),
// and the other chirality is T^T = J T J (J reverses s).  The hop results are
// transposed through LDS so that one lane holds one spin-colour component of
// a site for every s (components of the transposed chirality stored in
// reversed s order), applies T from registers with uniform coefficients, and
// transposes back: four LDS passes of one spinor per lane instead of Ls.
//
// Reductions: RED = 1 writes per-workgroup partials of |out|^2; RED = 2 is the
// conjugate-gradient residual update out = out - alpha * result (alpha read
// from device memory) with partials of the updated |out|^2.
#include "dwf_common.h"

namespace dwf {

struct StencilKArgs {
    Field in, self, out;
    const void *links;  // output-parity links [vh][8][9]
    const int *nbr;     // output-parity neighbours [vh][8]
    long vh;
    int Ls;
    int run;
    const void *emat;   // [2][Ls][Ls] in the arithmetic type (dense epilogue)
    double e0, e1, s0, s1, mf, sigma, tau;
    int edag, sdag;
    double *partial;
    long bstride;  // bytes between batch members (blockIdx.y), 0 for one field
    double tcoef[32];      // Toeplitz epilogue: f_k (k < Ls), then -mf f_k
    int trev;              // Toeplitz epilogue: P+ components use reversed s order
    int trat;              // Toeplitz epilogue in rational form, coefficients rcoef:
    double rcoef[24];      //   [0] y0 scale, [k] -mf r^k (1 <= k < Ls), [16] eps, [17] 1/delta,
                           //   [18] beta, [19] gamma, [20] -mf gamma
    const double *alpha;   // RED = 2: device pointer to alpha
};

// LDS rows of staged links: 72 entries per site padded to 73, so that the
// rows of the sites in a wavefront start in different banks; every entry of a
// row is then at a compile-time offset from the row start
constexpr int LK_STRIDE = 73;

// half-spinor projection h = upper pair of (1 + P g_MU) v
template <typename C, int MU, int P>
__device__ __forceinline__ void project(const cx<C> v[12], cx<C> h[6])
{
#pragma unroll
    for (int col = 0; col < 3; col++) {
        const cx<C> u0 = v[col], u1 = v[3 + col], l0 = v[6 + col], l1 = v[9 + col];
        if constexpr (MU == 0) {
            h[col] = (P > 0) ? u0 - timesI(l1) : u0 + timesI(l1);
            h[3 + col] = (P > 0) ? u1 - timesI(l0) : u1 + timesI(l0);
        } else if constexpr (MU == 1) {
            h[col] = (P > 0) ? u0 - l1 : u0 + l1;
            h[3 + col] = (P > 0) ? u1 + l0 : u1 - l0;
        } else if constexpr (MU == 2) {
            h[col] = (P > 0) ? u0 - timesI(l0) : u0 + timesI(l0);
            h[3 + col] = (P > 0) ? u1 + timesI(l1) : u1 - timesI(l1);
        } else {
            h[col] = (P > 0) ? u0 + l0 : u0 - l0;
            h[3 + col] = (P > 0) ? u1 + l1 : u1 - l1;
        }
    }
}

// f = sign(NEG) a.half[SA] + b.half[SB] in FP32 from two packed FP16 pairs,
// one v_fma_mix_f32 (a * 1.0 + b with both operands read as FP16); the sum of
// two FP16 numbers is formed exactly as in FP32 after conversion
template <int SA, int SB, bool NEG>
__device__ __forceinline__ float mix_add(uint32_t a, uint32_t b)
{
    float r;
#define DWF_MIX(STR) asm volatile(STR : "=v"(r) : "v"(a), "v"(b))
    if constexpr (!NEG && SA == 0 && SB == 0) DWF_MIX("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,1]");
    else if constexpr (!NEG && SA == 0 && SB == 1) DWF_MIX("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]");
    else if constexpr (!NEG && SA == 1 && SB == 0) DWF_MIX("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]");
    else if constexpr (!NEG && SA == 1 && SB == 1) DWF_MIX("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]");
    else if constexpr (NEG && SA == 0 && SB == 0) DWF_MIX("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,1]");
    else if constexpr (NEG && SA == 0 && SB == 1) DWF_MIX("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]");
    else if constexpr (NEG && SA == 1 && SB == 0) DWF_MIX("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]");
    else DWF_MIX("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]");
#undef DWF_MIX
    return r;
}

// the same projection on raw FP16 pairs (re in the low, im in the high half):
// with x = u + s l (s = +-1) or u + s i l, componentwise
//   u + s l   : (u.re + s l.re, u.im + s l.im)
//   u + s i l : (u.re - s l.im, u.im + s l.re)
template <int MU, int P>
__device__ __forceinline__ void project_f16(const uint32_t r[12], cx<float> h[6])
{
#pragma unroll
    for (int col = 0; col < 3; col++) {
        const uint32_t u0 = r[col], u1 = r[3 + col], l0 = r[6 + col], l1 = r[9 + col];
        if constexpr (MU == 0) {  // h0 = u0 - P i l1, h1 = u1 - P i l0
            h[col] = mk(mix_add<1, 0, (P < 0)>(l1, u0), mix_add<0, 1, (P > 0)>(l1, u0));
            h[3 + col] = mk(mix_add<1, 0, (P < 0)>(l0, u1), mix_add<0, 1, (P > 0)>(l0, u1));
        } else if constexpr (MU == 1) {  // h0 = u0 - P l1, h1 = u1 + P l0
            h[col] = mk(mix_add<0, 0, (P > 0)>(l1, u0), mix_add<1, 1, (P > 0)>(l1, u0));
            h[3 + col] = mk(mix_add<0, 0, (P < 0)>(l0, u1), mix_add<1, 1, (P < 0)>(l0, u1));
        } else if constexpr (MU == 2) {  // h0 = u0 - P i l0, h1 = u1 + P i l1
            h[col] = mk(mix_add<1, 0, (P < 0)>(l0, u0), mix_add<0, 1, (P > 0)>(l0, u0));
            h[3 + col] = mk(mix_add<1, 0, (P > 0)>(l1, u1), mix_add<0, 1, (P < 0)>(l1, u1));
        } else {  // h0 = u0 + P l0, h1 = u1 + P l1
            h[col] = mk(mix_add<0, 0, (P < 0)>(l0, u0), mix_add<1, 1, (P < 0)>(l0, u0));
            h[3 + col] = mk(mix_add<0, 0, (P < 0)>(l1, u1), mix_add<1, 1, (P < 0)>(l1, u1));
        }
    }
}

// acc += scale * (1 + P g_MU) U (projected h): the two colour vectors of h are
// multiplied by the link, the lower spin pair rebuilt from the upper one; the
// neighbour's FP16 site scale is applied in the accumulation
template <typename C, int MU, int P>
__device__ __forceinline__ void link_accumulate(cx<C> acc[12], const cx<C> h[6], const cx<C> u[9], bool first, C scale)
{
    cx<C> g[6];
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cx<C> t = cmul(u[r * 3 + 0], h[j * 3 + 0]);
            cmac(t, u[r * 3 + 1], h[j * 3 + 1]);
            cmac(t, u[r * 3 + 2], h[j * 3 + 2]);
            g[j * 3 + r] = t;
        }
    // lower pair: P i sigma_k g (k = x,y,z) or P g (t)
    cx<C> lo0[3], lo1[3];
#pragma unroll
    for (int col = 0; col < 3; col++) {
        const cx<C> g0 = g[col], g1 = g[3 + col];
        if constexpr (MU == 0) {
            lo0[col] = (P > 0) ? timesI(g1) : timesMinusI(g1);
            lo1[col] = (P > 0) ? timesI(g0) : timesMinusI(g0);
        } else if constexpr (MU == 1) {
            lo0[col] = (P > 0) ? g1 : -g1;
            lo1[col] = (P > 0) ? -g0 : g0;
        } else if constexpr (MU == 2) {
            lo0[col] = (P > 0) ? timesI(g0) : timesMinusI(g0);
            lo1[col] = (P > 0) ? timesMinusI(g1) : timesI(g1);
        } else {
            lo0[col] = (P > 0) ? g0 : -g0;
            lo1[col] = (P > 0) ? g1 : -g1;
        }
    }
    auto acc_add = [&](cx<C> &a, cx<C> b) {
        a.re = fma(scale, b.re, a.re);
        a.im = fma(scale, b.im, a.im);
    };
    if (first) {
#pragma unroll
        for (int col = 0; col < 3; col++) {
            acc[col] = scale * g[col];
            acc[3 + col] = scale * g[3 + col];
            acc[6 + col] = scale * lo0[col];
            acc[9 + col] = scale * lo1[col];
        }
    } else {
#pragma unroll
        for (int col = 0; col < 3; col++) {
            acc_add(acc[col], g[col]);
            acc_add(acc[3 + col], g[3 + col]);
            acc_add(acc[6 + col], lo0[col]);
            acc_add(acc[9 + col], lo1[col]);
        }
    }
}

// Buffer resources of an FP16 input field: the three 16-byte planes are read
// with one 32-bit lane offset and a scalar plane offset, so a neighbour load
// costs one integer multiply-add instead of 64-bit address arithmetic
struct InRsrc {
    __amdgpu_buffer_rsrc_t data, norm;
    int plane;  // bytes between planes
};

__device__ __forceinline__ InRsrc in_rsrc(const Field &f)
{
    // word 3 of the descriptor: raw (untyped) access on gfx9-class devices
    constexpr int kWord3 = 0x00020000;
    InRsrc r;
    r.plane = (int)(f.n * 16);
    r.data = __builtin_amdgcn_make_buffer_rsrc(f.data, 0, 3 * r.plane, kWord3);
    r.norm = __builtin_amdgcn_make_buffer_rsrc(f.norm, 0, (int)(f.n * 4), kWord3);
    return r;
}

// one direction of the hop; the workgroup's links and neighbour indices are in
// LDS: lk[j * LK_STRIDE + d * 9 + k], nbs[j * 8 + d]
template <typename S, typename C, int D, bool DAG>
__device__ __forceinline__ void hop_step(cx<C> acc[12], const StencilKArgs &a, const InRsrc &rs, const cx<C> *lk,
                                         const int *nbs, int j, int sb, int s)
{
    constexpr int MU = D & 3;
    constexpr int P0 = (D < 4) ? -1 : +1;
    constexpr int P = DAG ? -P0 : P0;
    const int nb = nbs[j * 8 + D];
    if (nb < 0) return;  // link across a Dirichlet face: zero contribution, no load
    cx<C> h[6];
    C scale;
    if constexpr (S::prec == P_F16) {
        const int i = nb * a.Ls + s;  // < 2^27 for fields below 2 GB
        uint32_t r[12];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const uint4 w =
                __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs.data, i * 16, q * rs.plane, 0));
            r[4 * q] = w.x;
            r[4 * q + 1] = w.y;
            r[4 * q + 2] = w.z;
            r[4 * q + 3] = w.w;
        }
        scale = C(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs.norm, i * 4, 0, 0)));
        project_f16<MU, P>(r, h);
    } else {
        const long i = (long)nb * a.Ls + s;
        cx<C> v[12];
        load_spinor_unscaled<S, C>(a.in, i, v, scale);
        project<C, MU, P>(v, h);
    }
    cx<C> u[9];
#pragma unroll
    for (int k = 0; k < 9; k++) u[k] = lk[j * LK_STRIDE + D * 9 + k];
    link_accumulate<C, MU, P>(acc, h, u, D == 0, scale);
}

// FP16 neighbour spinor as loaded: three 16-byte planes and the site scale
struct NbF16 {
    uint32_t r[12];
    float scale;
};

// Loads carry no branch, so the next direction's loads can be issued before
// this direction's arithmetic.  nb < 0 marks a link across a Dirichlet face:
// its offset is then placed beyond the buffer's range, where a buffer load
// returns zeros without a memory access, and the contribution vanishes with
// the zero scale.
__device__ __forceinline__ NbF16 load_nb_f16(const InRsrc &rs, int nb, int Ls, int s)
{
    constexpr int kOutOfRange = (int)0x80000000u;
    const int i = nb * Ls + s;  // < 2^27 for fields below 2 GB
    const int o16 = nb < 0 ? kOutOfRange : i * 16;
    const int o4 = nb < 0 ? kOutOfRange : i * 4;
    NbF16 v;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const uint4 w = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs.data, o16, q * rs.plane, 0));
        v.r[4 * q] = w.x;
        v.r[4 * q + 1] = w.y;
        v.r[4 * q + 2] = w.z;
        v.r[4 * q + 3] = w.w;
    }
    v.scale = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs.norm, o4, 0, 0));
    return v;
}

// the accumulator is materialised here: left free, the compiler may sink each
// direction's accumulation to the end and keep every direction's products live
template <typename C>
__device__ __forceinline__ void pin_acc(cx<C> acc[12])
{
#pragma unroll
    for (int c = 0; c < 12; c++) asm volatile("" : "+v"(acc[c].re), "+v"(acc[c].im));
}

// acc += scale * (1 + P g_MU) U h, one colour row of the link at a time: row
// r gives the colour-r entries of both projected spin vectors, and those alone
// feed the four accumulator entries of colour r (upper pair, and lower pair
// rebuilt), so only three link entries and two products are live at once.
// The arithmetic per output entry is that of link_accumulate.
template <typename C, int MU, int P>
__device__ __forceinline__ void link_accumulate_rows(cx<C> acc[12], const cx<C> h[6], const cx<C> *u, bool first,
                                                     C scale)
{
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const cx<C> u0 = u[r * 3 + 0], u1 = u[r * 3 + 1], u2 = u[r * 3 + 2];
        cx<C> g0 = cmul(u0, h[0]);
        cmac(g0, u1, h[1]);
        cmac(g0, u2, h[2]);
        cx<C> g1 = cmul(u0, h[3]);
        cmac(g1, u1, h[4]);
        cmac(g1, u2, h[5]);
        cx<C> lo0, lo1;
        if constexpr (MU == 0) {
            lo0 = (P > 0) ? timesI(g1) : timesMinusI(g1);
            lo1 = (P > 0) ? timesI(g0) : timesMinusI(g0);
        } else if constexpr (MU == 1) {
            lo0 = (P > 0) ? g1 : -g1;
            lo1 = (P > 0) ? -g0 : g0;
        } else if constexpr (MU == 2) {
            lo0 = (P > 0) ? timesI(g0) : timesMinusI(g0);
            lo1 = (P > 0) ? timesMinusI(g1) : timesI(g1);
        } else {
            lo0 = (P > 0) ? g0 : -g0;
            lo1 = (P > 0) ? g1 : -g1;
        }
        if (first) {
            acc[r] = scale * g0;
            acc[3 + r] = scale * g1;
            acc[6 + r] = scale * lo0;
            acc[9 + r] = scale * lo1;
        } else {
            acc[r].re = fma(scale, g0.re, acc[r].re);
            acc[r].im = fma(scale, g0.im, acc[r].im);
            acc[3 + r].re = fma(scale, g1.re, acc[3 + r].re);
            acc[3 + r].im = fma(scale, g1.im, acc[3 + r].im);
            acc[6 + r].re = fma(scale, lo0.re, acc[6 + r].re);
            acc[6 + r].im = fma(scale, lo0.im, acc[6 + r].im);
            acc[9 + r].re = fma(scale, lo1.re, acc[9 + r].re);
            acc[9 + r].im = fma(scale, lo1.im, acc[9 + r].im);
        }
    }
}

template <typename C, int D, bool DAG>
__device__ __forceinline__ void hop_f16(cx<C> acc[12], const NbF16 &v, const cx<C> *lk, int j)
{
    constexpr int MU = D & 3;
    constexpr int P0 = (D < 4) ? -1 : +1;
    constexpr int P = DAG ? -P0 : P0;
    cx<C> h[6];
    project_f16<MU, P>(v.r, h);
    link_accumulate_rows<C, MU, P>(acc, h, lk + j * LK_STRIDE + D * 9, D == 0, C(v.scale));
    pin_acc<C>(acc);
}

// the eight directions of the FP16 hop, loads running one direction ahead;
// the scheduling barriers keep that order (left free, the scheduler may hoist
// all eight loads and trade most of the occupancy for them)
template <typename C, bool DAG>
__device__ __forceinline__ void hop_f16_all(cx<C> acc[12], const InRsrc &rs, const cx<C> *lk, const int *nbs, int j,
                                            int Ls, int s)
{
    const int *nj = nbs + j * 8;
    NbF16 v[2];
    v[0] = load_nb_f16(rs, nj[0], Ls, s);
#define DWF_HOP_STAGE(D)                                               \
    if constexpr (D < 7) v[(D + 1) & 1] = load_nb_f16(rs, nj[D + 1], Ls, s); \
    __builtin_amdgcn_sched_barrier(0);                                 \
    hop_f16<C, D, DAG>(acc, v[D & 1], lk, j);                          \
    __builtin_amdgcn_sched_barrier(0);
    DWF_HOP_STAGE(0)
    DWF_HOP_STAGE(1)
    DWF_HOP_STAGE(2)
    DWF_HOP_STAGE(3)
    DWF_HOP_STAGE(4)
    DWF_HOP_STAGE(5)
    DWF_HOP_STAGE(6)
    DWF_HOP_STAGE(7)
#undef DWF_HOP_STAGE
}

// cooperative load of the links and neighbour indices of the sb consecutive
// internal sites from base into LDS (each link read once per workgroup
// instead of once per lane).  Both tables are site-major, so the workgroup's
// entries are one contiguous block: it is read in 16-byte pieces spread over
// all lanes, and every piece of a round is requested before any is used.
template <typename S, typename C>
__device__ __forceinline__ void stage_links(const StencilKArgs &a, long base, int sb, cx<C> *lk, int *nbs)
{
    using P = Planes<S>;              // complex entries per 16-byte piece
    constexpr int CPS = 72 / P::cpp;  // pieces per site
    constexpr int R = 4;              // pieces per lane and round
    const int nt = blockDim.x * blockDim.y;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const long left = a.vh - base;
    const int ns = left < sb ? (int)left : sb;  // sites of the workgroup inside the field
    const int npc = ns * CPS;
    // the block is read by this workgroup alone: non-temporal loads
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const uint4 *src = (const uint4 *)a.links + base * CPS;
    for (int c0 = tid; c0 < npc; c0 += R * nt) {
        uint4 w[R];
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int c = c0 + k * nt;
            if (c < npc) w[k] = __builtin_bit_cast(uint4, __builtin_nontemporal_load((const v4u *)(src + c)));
        }
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int c = c0 + k * nt;
            if (c < npc) {
                const int site = c / CPS, e0 = (c - site * CPS) * P::cpp;
                Vec16 v;
                v.u = w[k];
#pragma unroll
                for (int e = 0; e < P::cpp; e++) {
                    if constexpr (LinkQ15<S>::value)
                        lk[site * LK_STRIDE + e0 + e] = unpack_q15<C>(((const uint32_t *)&v.u)[e]);
                    else
                        lk[site * LK_STRIDE + e0 + e] = unpack<C>(vec_get<S>(v, e));
                }
            }
        }
    }
    // eight indices per site: two 16-byte pieces, landing at nbs[site * 8 + d]
    const int4 *nsrc = (const int4 *)a.nbr + base * 2;
    for (int c = tid; c < 2 * ns; c += nt) {
        const int4 v = nsrc[c];
        nbs[4 * c] = v.x;
        nbs[4 * c + 1] = v.y;
        nbs[4 * c + 2] = v.z;
        nbs[4 * c + 3] = v.w;
    }
}

// batch member blockIdx.y of fields laid out `stride` bytes apart
__device__ __forceinline__ Field batch_member(Field f, long stride)
{
    if (stride) {
        const long off = (long)blockIdx.y * stride;
        f.data = (char *)f.data + off;
        if (f.norm) f.norm = (float *)((char *)f.norm + off);
    }
    return f;
}

// byte offset of the self-input region in LDS: behind the staged links and
// behind the epilogue's hop results (and dense matrix), which alias the links
template <typename C>
__host__ __device__ inline size_t stencil_self_offset(int epi, int sb, int Ls, int lsc)
{
    const size_t links = (size_t)sb * (73 * sizeof(cx<C>) + 8 * sizeof(int));
    size_t epil = 0;
    if (epi == EPI_TOEP) epil = (size_t)sb * 12 * (lsc * sizeof(cx<C>) + 16);
    else if (epi != EPI_NONE) epil = (size_t)sb * Ls * 12 * sizeof(cx<C>);
    if (epi == EPI_DENSE) epil += 2 * (size_t)Ls * Ls * sizeof(C);
    return ((links > epil ? links : epil) + 15) & ~(size_t)15;
}

// o = T a for the twisted-circulant T of first column f (g = -mf f)
template <typename C, int LSC>
__device__ __forceinline__ void toeplitz_apply(const cx<C> av[LSC], cx<C> o[LSC], const C f[LSC], const C g[LSC])
{
#pragma unroll
    for (int t = 0; t < LSC; t++) {
        cx<C> v = mk(C(0), C(0));
#pragma unroll
        for (int k = 0; k < LSC; k++) {
            const C w = (k <= t) ? f[k] : g[k];
            const cx<C> x = (k <= t) ? av[t - k] : av[t - k + LSC];
            v.re = fma(w, x.re, v.re);
            v.im = fma(w, x.im, v.im);
        }
        o[t] = v;
    }
}

// o = T a for T = (beta + gamma S)(delta + eps S)^-1 (the same twisted-circulant
// operator in O(Ls)): y = (delta + eps S)^-1 a from its first entry
//   y_0 = (a_0 - mf sum_{k>=1} r^k a_{Ls-k}) / (delta (1 + mf r^Ls)),  r = -eps/delta,
// and the rows delta y_t + eps y_{t-1} = a_t; then o_t = beta y_t + gamma y_{t-1}
// with the twisted wrap for t = 0
template <typename C, int LSC>
__device__ __forceinline__ void toeplitz_rational(const cx<C> av[LSC], cx<C> o[LSC], const double *rc)
{
    cx<C> y0 = av[0];
#pragma unroll
    for (int k = 1; k < LSC; k++) {
        const C w = C(rc[k]);
        y0.re = fma(w, av[LSC - k].re, y0.re);
        y0.im = fma(w, av[LSC - k].im, y0.im);
    }
    const C ep = C(rc[16]), idl = C(rc[17]), be = C(rc[18]), ga = C(rc[19]), gw = C(rc[20]);
    cx<C> y[LSC];
    y[0] = C(rc[0]) * y0;
#pragma unroll
    for (int t = 1; t < LSC; t++) {
        y[t].re = idl * fma(-ep, y[t - 1].re, av[t].re);
        y[t].im = idl * fma(-ep, y[t - 1].im, av[t].im);
    }
    o[0].re = fma(be, y[0].re, gw * y[LSC - 1].re);
    o[0].im = fma(be, y[0].im, gw * y[LSC - 1].im);
#pragma unroll
    for (int t = 1; t < LSC; t++) {
        o[t].re = fma(be, y[t].re, ga * y[t - 1].re);
        o[t].im = fma(be, y[t].im, ga * y[t - 1].im);
    }
}

template <typename S, typename C, int EPI, bool SELF, bool DAG, int RED, int LSC>
__global__ void __launch_bounds__(256) k_stencil(StencilKArgs a)
{
    a.in = batch_member(a.in, a.bstride);
    a.out = batch_member(a.out, a.bstride);
    if constexpr (SELF) a.self = batch_member(a.self, a.bstride);
    const int Ls = a.Ls;
    const int s = threadIdx.x;
    const int j = threadIdx.y;
    const int sb = blockDim.y;
    const int tile = xcd_swizzle(blockIdx.x, gridDim.x, a.run);
    const long cb = (long)tile * sb + j;
    const bool valid = cb < a.vh;
    const long i = cb * Ls + s;

    // LDS: staged links + neighbour indices during the hop, reused afterwards
    // by the epilogue (hop results, dense matrix); the self input has its own
    // region behind both, filled before the hop (stencil_lds_bytes)
    extern __shared__ unsigned char smem[];
    cx<C> *lk = (cx<C> *)smem;
    int *nbs = (int *)(lk + LK_STRIDE * sb);
    cx<C> *lds_h = (cx<C> *)smem;
    C *lds_e = (C *)(lds_h + sb * Ls * 12);
    cx<C> *lds_s = (cx<C> *)(smem + stencil_self_offset<C>(EPI, sb, Ls, LSC));

    if constexpr (SELF) {
        // the self input goes to LDS before the hop: its load overlaps the link
        // staging and the hop, and it holds no registers during the hop
        cx<C> own[12];
        if (valid) {
            load_spinor<S, C>(a.self, i, own);
        } else {
#pragma unroll
            for (int c = 0; c < 12; c++) own[c] = mk(C(0), C(0));
        }
        cx<C> *bs = lds_s + j * 12 * Ls + s;  // component-major rows [c][s]
#pragma unroll
        for (int c = 0; c < 12; c++) bs[c * Ls] = own[c];
    }
    // residual of the fused CG update: issued now, used after the hop
    // (16-bit storage only; wider formats would hold too many registers)
    constexpr bool PRE_R = RED == 2 && sizeof(typename S::elem) == 4;
    RawSpinor<S> r_raw;
    if constexpr (PRE_R) {
        if (valid) load_raw<S>(a.out, i, r_raw);
    }
    stage_links<S, C>(a, (long)tile * sb, sb, lk, nbs);
    __syncthreads();
    cx<C> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = mk(C(0), C(0));
    InRsrc rs{};
    if constexpr (S::prec == P_F16) rs = in_rsrc(a.in);
    if constexpr (S::prec == P_F16) {
        if (valid) hop_f16_all<C, DAG>(acc, rs, lk, nbs, j, Ls, s);
    } else if (valid) {
        hop_step<S, C, 0, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 1, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 2, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 3, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 4, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 5, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 6, DAG>(acc, a, rs, lk, nbs, j, sb, s);
        hop_step<S, C, 7, DAG>(acc, a, rs, lk, nbs, j, sb, s);
    }
    if constexpr (EPI != EPI_NONE) __syncthreads();  // the staged links are dead from here
    const C mf = C(a.mf);
    cx<C> res[12];
    const C tau = C(a.tau);
    if constexpr (EPI == EPI_TOEP) {
        static_assert(!SELF && LSC > 0 && LSC <= 16, "Toeplitz epilogue: no self term, 1 <= Ls <= 16");
        // rows [site j][component c] of LSC values, padded by 16 bytes against bank conflicts
        constexpr int RS = LSC + 16 / (int)sizeof(cx<C>);
        cx<C> *rows = lds_h + j * 12 * RS;
        const bool rp = a.trev != 0;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const bool rev = (c < 6) ? rp : !rp;
            rows[c * RS + (rev ? LSC - 1 - s : s)] = acc[c];
        }
        __syncthreads();
        C f[LSC], g[LSC];
#pragma unroll
        for (int k = 0; k < LSC; k++) {
            f[k] = C(a.tcoef[k]);
            g[k] = C(a.tcoef[16 + k]);
        }
        for (int c = s; c < 12; c += LSC) {
            cx<C> av[LSC], o[LSC];
#pragma unroll
            for (int t = 0; t < LSC; t++) av[t] = rows[c * RS + t];
            if (a.trat)
                toeplitz_rational<C, LSC>(av, o, a.rcoef);
            else
                toeplitz_apply<C, LSC>(av, o, f, g);
#pragma unroll
            for (int t = 0; t < LSC; t++) rows[c * RS + t] = o[t];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const bool rev = (c < 6) ? rp : !rp;
            res[c] = tau * rows[c * RS + (rev ? LSC - 1 - s : s)];
        }
    } else {
        if constexpr (EPI != EPI_NONE) {
            cx<C> *bh = lds_h + j * 12 * Ls + s;  // component-major rows [c][s]
#pragma unroll
            for (int c = 0; c < 12; c++) bh[c * Ls] = acc[c];
            if constexpr (EPI == EPI_DENSE) {
                const C *em = (const C *)a.emat;
                const int tid = threadIdx.x + blockDim.x * threadIdx.y;
                for (int k = tid; k < 2 * Ls * Ls; k += blockDim.x * blockDim.y) lds_e[k] = em[k];
            }
            __syncthreads();
        }
        if constexpr (EPI == EPI_NONE) {
#pragma unroll
            for (int c = 0; c < 12; c++) res[c] = tau * acc[c];
        } else if constexpr (EPI == EPI_DENSE) {
            const cx<C> *blk = lds_h + j * 12 * Ls;
            const C *Mu = lds_e + s * Ls;            // P+ block row s
            const C *Ml = lds_e + Ls * Ls + s * Ls;  // P- block row s
#pragma unroll
            for (int c = 0; c < 12; c++) res[c] = mk(C(0), C(0));
            for (int t = 0; t < Ls; t++) {
                const C mu = Mu[t], ml = Ml[t];
#pragma unroll
                for (int c = 0; c < 12; c++) {
                    const C m = (c < 6) ? mu : ml;
                    const cx<C> v = blk[c * Ls + t];
                    res[c].re = fma(m, v.re, res[c].re);
                    res[c].im = fma(m, v.im, res[c].im);
                }
            }
#pragma unroll
            for (int c = 0; c < 12; c++) res[c] = tau * res[c];
        } else {
            const cx<C> *blk = lds_h + j * 12 * Ls;
            const C e0 = C(a.e0), e1 = C(a.e1);
#pragma unroll
            for (int c = 0; c < 12; c++) res[c] = tau * (e0 * acc[c] + e1 * shift5t<C>(blk, c, s, Ls, a.edag, mf));
        }
        if constexpr (SELF) {
            const cx<C> *blk = lds_s + j * 12 * Ls;
            const C s0 = C(a.s0), s1 = C(a.s1), sg = C(a.sigma);
#pragma unroll
            for (int c = 0; c < 12; c++)
                res[c] = res[c] + sg * (s0 * blk[c * Ls + s] + s1 * shift5t<C>(blk, c, s, Ls, a.sdag, mf));
        }
    }
    if constexpr (RED == 2) {
        // conjugate-gradient residual update: out holds r on entry
        const C al = C(*a.alpha);
        if (valid) {
            cx<C> rv[12];
            if constexpr (PRE_R) unpack_raw<S, C>(r_raw, rv);
            else load_spinor<S, C>(a.out, i, rv);
#pragma unroll
            for (int c = 0; c < 12; c++) res[c] = rv[c] - al * res[c];
        }
    }
    if (valid) store_spinor<S, C, true>(a.out, i, res);
    // the reduction sees the field as stored (storage rounding applied)
    if constexpr (RED != 0) storage_round<S, C>(res);
    if constexpr (RED != 0) {
        double n2 = 0;
        if (valid) {
#pragma unroll
            for (int c = 0; c < 12; c++) n2 += double(res[c].re) * double(res[c].re) + double(res[c].im) * double(res[c].im);
        }
        const double t = block_sum(n2);
        if (threadIdx.x == 0 && threadIdx.y == 0) a.partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// s-local dense operator out = M in, M = [2][Ls][Ls] (P+ block, P- block)
template <typename S, typename C>
__global__ void __launch_bounds__(256) k_slocal(Field in, Field out, const C *mat, long vh, int Ls, int run, long bstride)
{
    in = batch_member(in, bstride);
    out = batch_member(out, bstride);
    const int s = threadIdx.x, j = threadIdx.y, sb = blockDim.y;
    const long cb = (long)xcd_swizzle(blockIdx.x, gridDim.x, run) * sb + j;
    const bool valid = cb < vh;
    const long i = cb * Ls + s;
    extern __shared__ unsigned char smem[];
    cx<C> *lds = (cx<C> *)smem;
    C *lm = (C *)(lds + sb * Ls * 12);
    cx<C> v[12];
    if (valid) {
        load_spinor<S, C>(in, i, v);
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = mk(C(0), C(0));
    }
#pragma unroll
    for (int c = 0; c < 12; c++) lds[(j * Ls + s) * 12 + c] = v[c];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    for (int k = tid; k < 2 * Ls * Ls; k += blockDim.x * blockDim.y) lm[k] = mat[k];
    __syncthreads();
    cx<C> res[12];
#pragma unroll
    for (int c = 0; c < 12; c++) res[c] = mk(C(0), C(0));
    const cx<C> *blk = lds + j * Ls * 12;
    for (int t = 0; t < Ls; t++) {
        const C mu = lm[s * Ls + t], ml = lm[Ls * Ls + s * Ls + t];
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const C m = (c < 6) ? mu : ml;
            res[c].re = fma(m, blk[t * 12 + c].re, res[c].re);
            res[c].im = fma(m, blk[t * 12 + c].im, res[c].im);
        }
    }
    if (valid) store_spinor<S, C>(out, i, res);
}

}  // namespace dwf

// ------------------------------------------------------------ host launchers
#include <cmath>

#include "dwf_internal.h"

namespace dwf {

template <typename S, typename C>
static int launch_stencil_t(Context &c, const StencilSpec &sp, Field in, Field self, Field out)
{
    const int Ls = c.Ls;
    // a dense epilogue whose operator is twisted-circulant runs as the Toeplitz epilogue
    int epi = sp.epi;
    const bool toep = epi == EPI_DENSE && sp.epi_op >= 0 && sp.epi_op < SL_NOP && c.toep_ok[sp.epi_op] &&
                      (Ls == 8 || Ls == 12 || Ls == 16) && !sp.self && !sp.reduce && !sp.cg_update;
    if (toep) epi = EPI_TOEP;
    auto lds_of = [&](int sb_) {
        return stencil_self_offset<C>(epi, sb_, Ls, epi == EPI_TOEP ? Ls : 0) +
               (sp.self ? (size_t)sb_ * Ls * 12 * sizeof(cx<C>) : 0);
    };
    // the schedule's sites per workgroup, halved while the LDS would not fit
    const LaunchCfg &cfg = sp.nbatch > 1 ? c.cfg_stencil_batch : c.cfg_stencil;
    int sb = cfg_sb(c, cfg);
    while (sb > 1 && lds_of(sb) > c.lds_max) sb = (sb + 1) / 2;
    const size_t lds = lds_of(sb);
    if (lds > c.lds_max) fail(DWF_ENOTSUP, "fifth dimension too long for the fused stencil's LDS");
    const long nblk = (c.vh + sb - 1) / sb;
    const int nb = std::max(1, sp.nbatch);
    if (sp.reduce && nblk * nb > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
    StencilKArgs a;
    a.bstride = nb > 1 ? sp.bstride : 0;
    a.in = in;
    a.self = self;
    a.out = out;
    a.links = c.links[S::prec][sp.out_parity];
    a.nbr = c.nbr_sm + (long)sp.out_parity * 8 * c.vh;
    a.vh = c.vh;
    a.Ls = Ls;
    a.run = cfg.run;
    a.emat = (epi == EPI_DENSE) ? slmat(c, sp.epi_op, sizeof(C) == 8) : nullptr;
    if (toep) {
        for (int k = 0; k < 16; k++) {
            a.tcoef[k] = k < Ls ? c.toep_f[sp.epi_op][k] : 0.0;
            a.tcoef[16 + k] = k < Ls ? -c.p.mf * c.toep_f[sp.epi_op][k] : 0.0;
        }
        a.trev = c.toep_rev[sp.epi_op];
        a.trat = c.toep_rat[sp.epi_op] ? 1 : 0;
        for (double &t : a.rcoef) t = 0.0;
        if (a.trat) {
            const double *q = c.toep_rc[sp.epi_op];
            const double mf = c.p.mf, r = -q[3] / q[2];
            a.rcoef[0] = 1.0 / (q[2] * (1.0 + mf * std::pow(r, Ls)));
            for (int k = 1; k < Ls; k++) a.rcoef[k] = -mf * std::pow(r, k);
            a.rcoef[16] = q[3];
            a.rcoef[17] = 1.0 / q[2];
            a.rcoef[18] = q[0];
            a.rcoef[19] = q[1];
            a.rcoef[20] = -mf * q[1];
        }
    } else {
        for (double &t : a.tcoef) t = 0.0;
        for (double &t : a.rcoef) t = 0.0;
        a.trev = 0;
        a.trat = 0;
    }
    a.alpha = sp.cg_update ? c.dscal + sp.alpha_slot : nullptr;
    if (sp.cg_update && (sp.alpha_slot < 0 || !sp.reduce)) fail(DWF_EINVAL, "residual update needs alpha and reduce");
    a.e0 = sp.e0;
    a.e1 = sp.e1;
    a.s0 = sp.s0;
    a.s1 = sp.s1;
    a.mf = c.p.mf;
    a.sigma = sp.sigma;
    a.tau = sp.tau;
    a.edag = sp.edag;
    a.sdag = sp.sdag;
    a.partial = c.partials;
    dim3 blk(Ls, sb), grid((unsigned)nblk, (unsigned)nb);
    // algorithmic traffic: neighbour spinor, 8 links shared by the Ls slices,
    // output, self input, residual input of the fused update
    const double sbytes = 12.0 * sizeof(typename S::elem) + (S::has_norm ? 4.0 : 0.0);
    const double bytes =
        nb * ((double)c.n5h * (2 * sbytes + (sp.self ? sbytes : 0.0) + (sp.cg_update ? sbytes : 0.0)) +
              (double)c.vh * 8 * 9 * sizeof(typename S::elem));
    double flops = nb * (double)c.n5h * 1320.0;
    if (sp.epi == EPI_DENSE) flops += nb * (double)c.n5h * 24.0 * 2.0 * Ls;
    Timer tm(c, sp.kclass, bytes, flops, S::prec);
    const int red = sp.cg_update ? 2 : (sp.reduce ? 1 : 0);
#define DWF_K(E, SF, DG, RD, LS) hipLaunchKernelGGL((k_stencil<S, C, E, SF, DG, RD, LS>), grid, blk, lds, c.stream, a)
#define DWF_DG(E, SF, RD, LS)        \
    if (sp.dagger)                   \
        DWF_K(E, SF, true, RD, LS);  \
    else                             \
        DWF_K(E, SF, false, RD, LS);
    bool done = true;
    if (epi == EPI_TOEP) {
        if (Ls == 8) {
            DWF_DG(EPI_TOEP, false, 0, 8)
        } else if (Ls == 12) {
            DWF_DG(EPI_TOEP, false, 0, 12)
        } else {
            DWF_DG(EPI_TOEP, false, 0, 16)
        }
    } else if (epi == EPI_NONE) {
        if (sp.self) {
            if (red == 1) {
                DWF_DG(EPI_NONE, true, 1, 0)
            } else if (red == 0) {
                DWF_DG(EPI_NONE, true, 0, 0)
            } else {
                done = false;
            }
        } else {
            if (red == 1) {
                DWF_DG(EPI_NONE, false, 1, 0)
            } else if (red == 0) {
                DWF_DG(EPI_NONE, false, 0, 0)
            } else {
                done = false;
            }
        }
    } else if (epi == EPI_DENSE) {
        if (!sp.self && red == 0) {
            DWF_DG(EPI_DENSE, false, 0, 0)
        } else {
            done = false;
        }
    } else if (epi == EPI_SHIFT && sp.self) {
        if (red == 2) {
            DWF_DG(EPI_SHIFT, true, 2, 0)
        } else if (red == 1) {
            DWF_DG(EPI_SHIFT, true, 1, 0)
        } else {
            DWF_DG(EPI_SHIFT, true, 0, 0)
        }
    } else {
        done = false;
    }
#undef DWF_DG
#undef DWF_K
    if (!done) fail(DWF_EINVAL, "unsupported fused stencil stage");
    HIPCHECK(hipGetLastError());
    return sp.reduce ? (int)nblk : 0;
}

template <typename S, typename C>
static void launch_slocal_t(Context &c, int op, Field in, Field out, int nbatch, long bstride)
{
    const int Ls = c.Ls;
    const int sb = cfg_sb(c, c.cfg_slocal);
    const long nblk = (c.vh + sb - 1) / sb;
    const int nb = std::max(1, nbatch);
    const size_t lds = (size_t)sb * Ls * 12 * sizeof(cx<C>) + 2 * (size_t)Ls * Ls * sizeof(C);
    const double sbytes = 12.0 * sizeof(typename S::elem) + (S::has_norm ? 4.0 : 0.0);
    Timer tm(c, DWF_K_SLOCAL, nb * 2.0 * sbytes * c.n5h, nb * (double)c.n5h * 48.0 * Ls, S::prec);
    hipLaunchKernelGGL((k_slocal<S, C>), dim3((unsigned)nblk, (unsigned)nb), dim3(Ls, sb), lds, c.stream, in, out,
                       (const C *)slmat(c, op, sizeof(C) == 8), c.vh, Ls, c.cfg_slocal.run, nb > 1 ? bstride : 0L);
    HIPCHECK(hipGetLastError());
}

}  // namespace dwf
