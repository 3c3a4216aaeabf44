// Gauge-equivariant parallel-transport convolution (PTC) network kernels.
//
// A layer maps Cin colour-vector channels to Cout:
//   out_a(x,s) = sum_pi sum_b W[pi][a][b] (T_pi phi_b)(x,s)
// over 11 paths pi: 0 identity; 1+mu: U_mu(x) phi(x+mu); 5+mu: U_mu(x-mu)^+ phi(x-mu);
// 9: phi(x,s+1) and 10: phi(x,s-1), zero outside 0 <= s < Ls.  The map is
// linear, commutes with local SU(3) rotations, and its adjoint is the same
// layer with W[pi]^+ on the adjoint path (T_{+mu}^+ = T_{-mu}, T_{+s}^+ = T_{-s}).
//
// Features are FP32 complex planes over both parities:
//   f[p][ch*3 + colour][i],  i = j*Ls + s (internal site order)
// Weights are BF16 (re, im) pairs converted to FP32 in LDS; all arithmetic FP32,
// weight-gradient partial sums FP64.
#include <type_traits>

#include "dwf_internal.h"

namespace dwf {

struct NetGeo {
    const int *nbr;        // [2][8][vh]
    const float2 *links0;  // FP32 links, output parity 0: [8][9][vh]
    const float2 *links1;  // output parity 1
    const int *nbr_sm;     // [2][vh][8], site-major
    const float2 *lsm0;    // FP32 links, output parity 0, site-major: [vh][8][9]
    const float2 *lsm1;    // output parity 1
    long vh;
    int Ls;
};

__device__ __forceinline__ cx<float> c2(float2 v) { return mk(v.x, v.y); }

// path source for output site (j, s) of parity p: returns the 5D index in the
// source parity and whether the site exists (s-paths have open ends)
__device__ __forceinline__ bool path_source(const NetGeo &g, int p, int pi, long j, int s, long &src, int &sp)
{
    if (pi == 0) {
        src = j * g.Ls + s;
        sp = p;
        return true;
    }
    if (pi <= 8) {
        const int d = (pi <= 4) ? pi - 1 : pi - 1;  // 1..4 -> 0..3 (+mu), 5..8 -> 4..7 (-mu)
        const int nb = g.nbr[((long)p * 8 + d) * g.vh + j];
        src = (long)(nb < 0 ? 0 : nb) * g.Ls + s;
        sp = 1 - p;
        return nb >= 0;  // -1: link across a Dirichlet face (zero)
    }
    const int s2 = (pi == 9) ? s + 1 : s - 1;
    src = j * g.Ls + s2;
    sp = p;
    return s2 >= 0 && s2 < g.Ls;
}

template <int CIN>
__device__ __forceinline__ void transported(const NetGeo &g, const float2 *in, long n, int p, int pi, long j, int s,
                                            cx<float> t[CIN][3])
{
    long src;
    int sp;
    const bool ok = path_source(g, p, pi, j, s, src, sp);
    const float2 *base = in + (long)sp * CIN * 3 * n;
    if (!ok) {
#pragma unroll
        for (int b = 0; b < CIN; b++)
#pragma unroll
            for (int c = 0; c < 3; c++) t[b][c] = mk(0.f, 0.f);
        return;
    }
#pragma unroll
    for (int b = 0; b < CIN; b++)
#pragma unroll
        for (int c = 0; c < 3; c++) t[b][c] = c2(base[(b * 3 + c) * n + src]);
    if (pi >= 1 && pi <= 8) {
        const int d = pi - 1;
        const float2 *L = (p ? g.links1 : g.links0) + (long)d * 9 * g.vh + j;
        cx<float> u[9];
#pragma unroll
        for (int k = 0; k < 9; k++) u[k] = c2(L[k * g.vh]);
#pragma unroll
        for (int b = 0; b < CIN; b++) {
            cx<float> v0 = t[b][0], v1 = t[b][1], v2 = t[b][2];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                cx<float> a = cmul(u[r * 3 + 0], v0);
                cmac(a, u[r * 3 + 1], v1);
                cmac(a, u[r * 3 + 2], v2);
                t[b][r] = a;
            }
        }
    }
}

// one layer, output parity p.  w: [11][COUT][CIN] BF16 pairs.  Only the paths
// in pmask (bit pi) are evaluated: the caller leaves out paths whose sources
// are known to be zero.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_ptc_fwd(NetGeo g, const float2 *in, float2 *out, const __hip_bfloat162 *w, int p,
                                                 long n, int pmask)
{
    __shared__ cx<float> W[11 * COUT * CIN];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    for (int k = tid; k < 11 * COUT * CIN; k += blockDim.x * blockDim.y) {
        const float2 f = __bfloat1622float2(w[k]);
        W[k] = mk(f.x, f.y);
    }
    __syncthreads();
    const int s = threadIdx.x;
    const long j = (long)blockIdx.x * blockDim.y + threadIdx.y;
    if (j >= g.vh) return;
    cx<float> acc[COUT][3];
#pragma unroll
    for (int a = 0; a < COUT; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[a][c] = mk(0.f, 0.f);
    for (int pi = 0; pi < 11; pi++) {
        if (!(pmask >> pi & 1)) continue;
        cx<float> t[CIN][3];
        transported<CIN>(g, in, n, p, pi, j, s, t);
        const cx<float> *Wp = W + pi * COUT * CIN;
#pragma unroll
        for (int a = 0; a < COUT; a++)
#pragma unroll
            for (int b = 0; b < CIN; b++) {
                const cx<float> wab = Wp[a * CIN + b];
#pragma unroll
                for (int c = 0; c < 3; c++) cmac(acc[a][c], wab, t[b][c]);
            }
    }
    float2 *o = out + (long)p * COUT * 3 * n;
    const long i = j * g.Ls + s;
#pragma unroll
    for (int a = 0; a < COUT; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) o[(a * 3 + c) * n + i] = make_float2(acc[a][c].re, acc[a][c].im);
}

// ------------------------------------------------- forward on the matrix cores
//
// For every output column (5D site, colour) a layer is out[a] = sum_q W_q[a] T_q
// with q = (path, input channel) and T_q the transported input: a complex GEMM
// of M = COUT, K = 11 CIN over all columns.  It runs in real form,
//   [Re out; Im out] = [[Wr, -Wi], [Wi, Wr]] [Re T; Im T],
// as 32 x 32 x 8 BF16 MFMA tiles with FP32 accumulation (rows m' = 2a + re/im,
// K index k' = 2q + re/im).  The transported inputs are built in FP32 on the
// vector units and rounded to BF16 for the B operand.  The weights are BF16
// already, so the A operand is exact; it is packed once per weight update in
// operand order [step][lane][4].

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A 4 -> 4 layer has 8 real rows: in a 32 x 32 tile 24 of the 32 rows, and 12
// of the 16 accumulators per lane, would hold nothing.  It runs as 16 x 16 x 16
// tiles instead (half the accumulator registers, so five wavefronts fit per
// SIMD instead of four with BF16 inputs), the K range of one path (8) in the
// lower half of the tile's 16 and zeros in the upper.
template <int CIN, int COUT>
constexpr bool kMfma16 = CIN == 4 && COUT == 4;

__device__ __forceinline__ short bf16_bits(float f)
{
    const __hip_bfloat16 h = __float2bfloat16(f);
    return *(const short *)&h;
}

// A operand of a CIN -> COUT layer: pk[(step * 64 + lane) * 4 + e] = A[m'][k'],
// m' = lane % 32, k' = 8 step + 4 (lane / 32) + e; for the 16 x 16 x 16 tiles
// m' = lane % 16, k' = 8 step + 4 (lane / 16) + e, zero for lane / 16 >= 2
template <int CIN, int COUT>
__global__ void k_pack_mfma_weights(const __hip_bfloat162 *w, short *pk)
{
    constexpr int NSTEP = 11 * CIN / 4;
    constexpr bool M16 = kMfma16<CIN, COUT>;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NSTEP * 64 * 4) return;
    const int e = t & 3, lane = (t >> 2) & 63, step = t >> 8;
    const int mr = M16 ? lane & 15 : lane & 31;
    const int kr = 8 * step + 4 * (M16 ? lane >> 4 : lane >> 5) + e;
    const int a = mr >> 1, rho = mr & 1, q = kr >> 1, sig = kr & 1;
    float v = 0.f;
    if (a < COUT && (!M16 || (lane >> 4) < 2)) {
        const int pi = q / CIN, b = q % CIN;
        const float2 wf = __bfloat1622float2(w[(pi * COUT + a) * CIN + b]);
        v = (rho == 0) ? (sig == 0 ? wf.x : -wf.y) : (sig == 0 ? wf.y : wf.x);
    }
    pk[t] = bf16_bits(v);
}

// One workgroup takes MF_S consecutive 5D sites, 32 per wavefront.  Per hop
// path, every lane transports the input channels of one of its wavefront's
// sites (two lanes per site, half the channels each): one link load, 3 x 3
// complex products per channel on the vector units, BF16 rounding, into the
// wavefront's LDS rows as B operand [channel pair][colour][site].  The
// wavefront then runs the path's MFMA steps on its three tiles (one per
// colour, 32 sites each).  The identity and the two fifth-dimension paths
// read the same sites of the output parity: they take one phase, from one
// load of the wavefront's sites and one halo site on either side.
static constexpr int MF_S = 128;

// feature element k of a plane array in FP32 pairs or BF16 pairs
template <bool BF>
__device__ __forceinline__ cx<float> ld_feat(const void *base, long k)
{
    if constexpr (BF) {
        const float2 f = __bfloat1622float2(((const __hip_bfloat162 *)base)[k]);
        return mk(f.x, f.y);
    } else {
        return c2(((const float2 *)base)[k]);
    }
}

// feature element from its raw load: a BF16 pair or an FP32 pair
template <bool BF>
__device__ __forceinline__ cx<float> raw_feat(typename std::conditional<BF, uint32_t, float2>::type r)
{
    if constexpr (BF) {
        return mk(__uint_as_float(r << 16), __uint_as_float(r & 0xffff0000u));
    } else {
        return c2(r);
    }
}

// Activations between layers may be BF16 (in_bf16 / out_bf16): the matrix
// cores round their B operand to BF16 anyway, and BF16 storage halves the bytes
// of the eleven path reads of every input channel.  The BF16 activations keep
// the two channels of a channel pair side by side,
//   f[p][pair*3 + colour][i] = (channel 2 pair, channel 2 pair + 1), 8 bytes,
// so that a lane reads both channels of a pair in one 8-byte load (the FP32
// features keep one plane per channel).
// Occupancy target: left free, the compiler puts the accumulators in AGPRs on
// top of the VGPRs and two waves per SIMD fit, too few to cover the per-path
// load latency.  With the accumulators in VGPRs, four waves fit without spills
// for CIN = 4 and three for wider inputs (whose prefetched features take more
// registers); five for the 4 -> 4 layer on its 16 x 16 tiles with BF16 input.
// io: bit 0 set: the input is an internal half spinor of the odd sites (the
// four spin channels of the network's embedded input, zero on the even sites),
// FP32 or (IBF) BF16, instead of features (first layer only); bits 1-2: the output is
// written as an internal half spinor of the odd sites, 1 in FP32 and 2 in BF16
// storage, instead of FP32 features (FP32 output of the last layer, p = 1 only).
// The conversions between spinor and feature layouts then need no pass of their own.
// BSP: the input is the BF16 odd half spinor (IBF, CIN = 4, io bit 0).
template <int CIN, int COUT, bool IBF, bool OBF, bool BSP = false>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(kMfma16<CIN, COUT> && IBF ? 5 : CIN <= 4 ? 4 : 3,
                                       kMfma16<CIN, COUT> && IBF ? 5 : CIN <= 4 ? 4 : 3))) k_ptc_fwd_mfma(NetGeo g, const void *in, void *out, const short *wpk, int p,
                                                      long n, int pmask, int io)
{
    static_assert(CIN % 4 == 0 && 2 * COUT <= 32, "channel counts");
    static_assert(!BSP || (IBF && CIN == 4), "the BF16 spinor input has four channels");
    constexpr int NP = CIN / 2, HP = NP / 2;
    // Each wavefront owns 32 of the workgroup's sites: its lanes transport
    // them (lane: site jc, half h of the channel pairs) and its matrix-core
    // tiles are their three colours, so the B operands a wavefront reads are
    // the ones it wrote, and the phases need no workgroup barrier.  LDS rows
    // [channel pair][colour] of CSW columns per wavefront: its 32 sites with
    // one halo site on either side (for the fifth-dimension paths).
    constexpr int CSW = 32 + 2, WREG = NP * 3 * CSW;
    constexpr int JMAX = MF_S / 8 + 2;  // 4D sites a workgroup spans when Ls >= 8
    __shared__ bf16x4 Tb[4 * WREG];
    __shared__ cx<float> lks[JMAX * 72];
    __shared__ int nbl[JMAX * 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, jc = lane & 31;
    const long i0 = (long)blockIdx.x * MF_S;
    bf16x4 *Tw = Tb + wave * WREG;
    // transport role: site ts, channel pairs [th HP, th HP + HP)
    const int ts = 32 * wave + jc, th = h;
    const long it = i0 + ts;
    const bool ok = it < n;
    const long j = ok ? it / g.Ls : 0;
    const int s = ok ? (int)(it - j * g.Ls) : 0;
    const bf16x4 *A = (const bf16x4 *)wpk + lane;
    // With Ls >= 8 the links and neighbour indices of the workgroup's 4D sites
    // (one contiguous block of each site-major table) are staged in LDS once,
    // instead of every lane loading them again for every path.
    const bool staged = g.Ls >= 8;
    const long j0 = i0 / g.Ls;
    const int jl = ok ? (int)(j - j0) : 0;  // local 4D site of this lane's transport role
    // accumulators: three 32 x 32 tiles (one per colour), or six 16 x 16 tiles
    // (colour, half of the wavefront's sites)
    constexpr bool M16 = kMfma16<CIN, COUT>;
    constexpr int NT = M16 ? 6 : 3, NR = M16 ? 4 : 16;
    using AccT = typename std::conditional<M16, f32x4, f32x16>::type;
    AccT acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int r = 0; r < NR; r++) acc[t][r] = 0.f;
    // Feature loads of a hop path are issued at the start of the previous
    // phase's matrix-core work, so they are in flight through it; only the
    // accumulators and operands are live there, so this costs no registers at
    // the peak (the transport phase).
    using RawT = typename std::conditional<IBF, uint32_t, float2>::type;
    // the thread's half `half` of the input channel pairs at 5D site src of
    // parity sp; returns whether the site holds data
    auto load = [&](long src, int sp, bool hv, int half, RawT (&rw)[HP][2][3]) -> bool {
        if constexpr (BSP) {
            // the BF16 odd half spinor: component ch * 3 + colour is word
            // (m & 3) of 16-byte plane m >> 2; channel pair (2 half,
            // 2 half + 1) is components 6 half .. 6 half + 5: a whole plane
            // and half of the middle one
            hv = hv && sp == 1;
            if (!hv) return false;
            const uint32_t *w = (const uint32_t *)in;
            uint32_t m[6];
            if (half == 0) {
                const uint4 a = *(const uint4 *)(w + 4 * src);
                const uint2 b = *(const uint2 *)(w + 4 * n + 4 * src);
                m[0] = a.x, m[1] = a.y, m[2] = a.z, m[3] = a.w, m[4] = b.x, m[5] = b.y;
            } else {
                const uint2 b = *(const uint2 *)(w + 4 * n + 4 * src + 2);
                const uint4 a = *(const uint4 *)(w + 8 * n + 4 * src);
                m[0] = b.x, m[1] = b.y, m[2] = a.x, m[3] = a.y, m[4] = a.z, m[5] = a.w;
            }
#pragma unroll
            for (int k = 0; k < 6; k++) rw[0][k / 3][k % 3] = m[k];
            return true;
        } else if constexpr (IBF) {
            // a uniform plane base and one 32-bit lane offset per load
            const uint32_t voff = (uint32_t)((src + (long)half * HP * 3 * n) * 8);
#pragma unroll
            for (int q = 0; q < HP; q++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const char *pb = (const char *)in + (long)(sp * NP * 3 + q * 3 + c) * n * 8;
                    if (hv) {
                        const uint2 w = *(const uint2 *)(pb + voff);
                        rw[q][0][c] = w.x;
                        rw[q][1][c] = w.y;
                    }
                }
        } else if (CIN == 4 && (io & 1)) {
            // the odd half spinor, component ch * 3 + colour in 16-byte planes of
            // two: channel pair (2 half, 2 half + 1) is components 6 half ..
            // 6 half + 5, whole planes 3 half .. 3 half + 2
            hv = hv && sp == 1;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if (!hv) continue;
                const float4 w = ((const float4 *)in)[(long)(3 * half + k) * n + src];
                const int m0 = 2 * k, m1 = 2 * k + 1;  // local components (channel e = m / 3, colour m % 3)
                rw[0][m0 / 3][m0 % 3] = make_float2(w.x, w.y);
                rw[0][m1 / 3][m1 % 3] = make_float2(w.z, w.w);
            }
        } else {
            const long base = (long)sp * CIN * 3 * n + src;
#pragma unroll
            for (int q = 0; q < HP; q++)
#pragma unroll
                for (int e = 0; e < 2; e++)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const long f = base + (long)((2 * (half * HP + q) + e) * 3 + c) * n;
                        if (hv) rw[q][e][c] = ((const RawT *)in)[f];
                    }
        }
        return hv;
    };
    RawT raw[HP][2][3];
    auto fetch = [&](int pi) -> bool {  // hop path pi (1..8) of this thread's transport role
        long src = 0;
        int sp = p;
        bool hv;
        if (staged) {
            const int nb = nbl[jl * 8 + pi - 1];
            src = (long)(nb < 0 ? 0 : nb) * g.Ls + s;
            sp = 1 - p;
            hv = ok && nb >= 0;
        } else {
            hv = ok && path_source(g, p, pi, j, s, src, sp);
        }
        return load(src, sp, hv, th, raw);
    };
    // transported (hop) or plain features of one site into LDS column col of
    // every colour, channel pairs of half `half`, rounded to BF16
    auto put = [&](const RawT (&rw)[HP][2][3], bool hv, bool hop, const cx<float> (&u)[9], int half, int col) {
#pragma unroll
        for (int q = 0; q < HP; q++) {
            const int pp = half * HP + q;
            cx<float> t[2][3];
#pragma unroll
            for (int e = 0; e < 2; e++) {
                if (hv) {
                    const cx<float> v0 = raw_feat<IBF>(rw[q][e][0]), v1 = raw_feat<IBF>(rw[q][e][1]),
                                    v2 = raw_feat<IBF>(rw[q][e][2]);
                    if (hop) {
#pragma unroll
                        for (int r = 0; r < 3; r++) {
                            t[e][r] = cmul(u[3 * r], v0);
                            cmac(t[e][r], u[3 * r + 1], v1);
                            cmac(t[e][r], u[3 * r + 2], v2);
                        }
                    } else {
                        t[e][0] = v0;
                        t[e][1] = v1;
                        t[e][2] = v2;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 3; r++) t[e][r] = mk(0.f, 0.f);
                }
            }
#pragma unroll
            for (int r = 0; r < 3; r++) {
                bf16x4 v;
                v[0] = bf16_bits(t[0][r].re);
                v[1] = bf16_bits(t[0][r].im);
                v[2] = bf16_bits(t[1][r].re);
                v[3] = bf16_bits(t[1][r].im);
                Tw[(pp * 3 + r) * CSW + col] = v;
            }
        }
    };
    // tile tt of this lane is colour tt of site ts (column jc); zup / zdn:
    // the site's s + 1 / s - 1 is past a wall
    const int sl = (int)((i0 + ts) % g.Ls);
    const bool zup = sl == g.Ls - 1, zdn = sl == 0;
    // shift 0: the column itself; +1 / -1: the fifth-dimension neighbour,
    // zero where it is past a wall
    // 16 x 16 tiles: lane column n16 (site 16 hf + n16 of the wavefront), K
    // group g16 (pair g16 of the path for g16 < 2, zeros above)
    const int n16 = lane & 15, g16 = lane >> 4;
    bool zup16[2] = {false, false}, zdn16[2] = {false, false};
    if constexpr (M16) {
#pragma unroll
        for (int hf = 0; hf < 2; hf++) {
            const int sl16 = (int)((i0 + 32 * wave + 16 * hf + n16) % g.Ls);
            zup16[hf] = sl16 == g.Ls - 1;
            zdn16[hf] = sl16 == 0;
        }
    }
    auto mfma_path = [&](int pi, int shift) {
        if constexpr (M16) {
            const bf16x4 a = A[pi * 64];
#pragma unroll
            for (int tt = 0; tt < 3; tt++)
#pragma unroll
                for (int hf = 0; hf < 2; hf++) {
                    bf16x4 b = {0, 0, 0, 0};
                    const bool zero = shift > 0 ? zup16[hf] : shift < 0 ? zdn16[hf] : false;
                    if (g16 < 2 && !zero) b = Tw[(g16 * 3 + tt) * CSW + 16 * hf + n16 + 1 + shift];
                    acc[2 * tt + hf] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[2 * tt + hf], 0, 0, 0);
                }
        } else {
            const bool zero = shift > 0 ? zup : shift < 0 ? zdn : false;
#pragma unroll
            for (int st = 0; st < CIN / 4; st++) {
                const bf16x4 a = A[(pi * (CIN / 4) + st) * 64];
#pragma unroll
                for (int tt = 0; tt < 3; tt++) {
                    bf16x4 b = Tw[((2 * st + h) * 3 + tt) * CSW + jc + 1 + shift];
                    if (zero) b = bf16x4{0, 0, 0, 0};
                    acc[tt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[tt], 0, 0, 0);
                }
            }
        }
    };
    // the wavefront's LDS writes are complete and ordered against its later
    // reads (LDS serves a wavefront's accesses in order; this keeps the
    // compiler from moving them across)
    auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // one element (channel pair pp, colour c) of a halo site of the output
    // parity, as a BF16 B operand entry
    auto halo = [&](long hs, int pp, int c) -> bf16x4 {
        bf16x4 v = {0, 0, 0, 0};
        if (hs < 0 || hs >= n) return v;
        if constexpr (IBF) {
            uint2 w;
            if constexpr (BSP) {
                if (p != 1) return v;  // the spinor holds the odd sites only
                const uint32_t *w32 = (const uint32_t *)in;
                const int m0 = 2 * pp * 3 + c, m1 = m0 + 3;  // components channel * 3 + colour
                w.x = w32[(long)(m0 >> 2) * 4 * n + 4 * hs + (m0 & 3)];
                w.y = w32[(long)(m1 >> 2) * 4 * n + 4 * hs + (m1 & 3)];
            } else {
                w = ((const uint2 *)in)[(long)p * NP * 3 * n + (long)(pp * 3 + c) * n + hs];
            }
            __builtin_memcpy(&v, &w, sizeof(v));
        } else {
            float2 f0, f1;
            if (CIN == 4 && (io & 1)) {
                if (p != 1) return v;  // the spinor holds the odd sites only
                const int m0 = 2 * pp * 3 + c, m1 = m0 + 3;  // components channel * 3 + colour
                f0 = ((const float2 *)in)[(long)(m0 >> 1) * 2 * n + 2 * hs + (m0 & 1)];
                f1 = ((const float2 *)in)[(long)(m1 >> 1) * 2 * n + 2 * hs + (m1 & 1)];
            } else {
                const long base = (long)p * CIN * 3 * n + hs;
                f0 = ((const float2 *)in)[base + (long)(2 * pp * 3 + c) * n];
                f1 = ((const float2 *)in)[base + (long)((2 * pp + 1) * 3 + c) * n];
            }
            v[0] = bf16_bits(f0.x);
            v[1] = bf16_bits(f0.y);
            v[2] = bf16_bits(f1.x);
            v[3] = bf16_bits(f1.y);
        }
        return v;
    };
    // Paths that read the output's own parity (identity, s + 1, s - 1) share
    // one load of the workgroup's sites plus one site on either side: their
    // B operands are the same LDS columns, shifted by one site for the
    // fifth-dimension paths.
    const int own = pmask & ((1 << 0) | (1 << 9) | (1 << 10));
    int hops = pmask & 0x1fe;  // hop paths still to run, in order (uniform over the workgroup)
    auto next_hop = [&]() -> int {
        if (!hops) return -1;
        const int q = __builtin_ctz(hops);
        hops &= hops - 1;
        return q;
    };
    // Phases: the own-parity paths (OWN) if any, then the hop paths.  One loop
    // with one matrix-core site keeps the accumulators in place.
    constexpr int OWN = 16;
    int cur = own ? OWN : next_hop();
    int pi_first = own ? next_hop() : -1;  // the hop that follows the own phase
    bool have = false;
    // the own-parity load is issued first, so that it is in flight while the
    // links are staged; launches without hop paths stage nothing
    if (cur == OWN) have = load(it, p, ok, th, raw);
    if (staged && (pmask & 0x1fe)) {
        const long ilast = (i0 + MF_S < n ? i0 + MF_S : n) - 1;
        const int nj = (int)(ilast / g.Ls - j0) + 1;
        const float2 *lsrc = (p ? g.lsm1 : g.lsm0) + j0 * 72;
        for (int k = tid; k < nj * 72; k += 256) lks[k] = c2(lsrc[k]);
        const int *nsrc = g.nbr_sm + ((long)p * g.vh + j0) * 8;
        for (int k = tid; k < nj * 8; k += 256) nbl[k] = nsrc[k];
        __syncthreads();
    }
    if (cur > 0 && cur != OWN) have = fetch(cur);
    const cx<float> unone[9] = {};
    while (cur > 0) {
        const bool ownph = cur == OWN;
        if (ownph) {
            // the two halo sites of this wavefront's 32: lane = (side, pair, colour)
            const int hk = lane % (NP * 3), hside = lane / (NP * 3);
            if (hside < 2)
                Tw[hk * CSW + (hside ? CSW - 1 : 0)] =
                    halo(hside ? i0 + 32 * wave + 32 : i0 + 32 * wave - 1, hk / 3, hk % 3);
            put(raw, have, false, unone, th, jc + 1);
        } else {
            cx<float> u[9];
            if (have) {
                if (staged) {
#pragma unroll
                    for (int k = 0; k < 9; k++) u[k] = lks[jl * 72 + (cur - 1) * 9 + k];
                } else {
                    const float2 *L = (p ? g.links1 : g.links0) + (long)(cur - 1) * 9 * g.vh + j;
#pragma unroll
                    for (int k = 0; k < 9; k++) u[k] = c2(L[(long)k * g.vh]);
                }
            }
            put(raw, have, true, u, th, jc + 1);
        }
        wave_sync();
        const int nxt = ownph ? pi_first : next_hop();
        const bool have_next = nxt > 0 ? fetch(nxt) : false;
        // the phase's paths, one at a time so that only one path's operands are live
        const int npath = ownph ? 3 : 1;
        for (int k = 0; k < npath; k++) {
            const int pk = ownph ? (k == 0 ? 0 : 8 + k) : cur;  // own: identity, s + 1, s - 1
            if (ownph && !(own >> pk & 1)) continue;
            mfma_path(pk, !ownph || k == 0 ? 0 : k == 1 ? 1 : -1);
        }
        wave_sync();
        have = have_next;
        cur = nxt;
    }
    // one channel pair (a0, a0 + 1) of colour cc at output site i
    auto store = [&](int a0, int cc, long i, float2 v0, float2 v1) {
        if constexpr (OBF) {
            const __hip_bfloat162 b0 = __float22bfloat162_rn(v0), b1 = __float22bfloat162_rn(v1);
            uint2 w;
            w.x = *(const uint32_t *)&b0;
            w.y = *(const uint32_t *)&b1;
            ((uint2 *)out)[(long)p * (COUT / 2) * 3 * n + (long)((a0 / 2) * 3 + cc) * n + i] = w;
        } else if (io >> 1 == 1) {
            // FP32 odd half spinor: 16-byte planes of two components
            const int c0 = a0 * 3 + cc, c1 = c0 + 3;
            ((float2 *)out)[(long)(c0 >> 1) * 2 * n + 2 * i + (c0 & 1)] = v0;
            ((float2 *)out)[(long)(c1 >> 1) * 2 * n + 2 * i + (c1 & 1)] = v1;
        } else if (io >> 1 == 2) {
            // BF16 odd half spinor: 16-byte planes of four components
            const int c0 = a0 * 3 + cc, c1 = c0 + 3;
            ((__hip_bfloat162 *)out)[(long)(c0 >> 2) * 4 * n + 4 * i + (c0 & 3)] = __float22bfloat162_rn(v0);
            ((__hip_bfloat162 *)out)[(long)(c1 >> 2) * 4 * n + 4 * i + (c1 & 3)] = __float22bfloat162_rn(v1);
        } else {
            const long k = (long)p * COUT * 3 * n + (long)(a0 * 3 + cc) * n + i;
            ((float2 *)out)[k] = v0;
            ((float2 *)out)[k + 3 * n] = v1;
        }
    };
    if constexpr (M16) {
        // accumulator register r of tile (tt, hf) holds row 4 g16 + r of column
        // n16: channels 2 g16 and 2 g16 + 1 (re, im each) of colour tt at site
        // 16 hf + n16 of the wavefront; rows 8 and up are zero
        if (g16 < 2) {
#pragma unroll
            for (int tt = 0; tt < 3; tt++)
#pragma unroll
                for (int hf = 0; hf < 2; hf++) {
                    const long i = i0 + 32 * wave + 16 * hf + n16;
                    if (i >= n) continue;
                    const AccT &v = acc[2 * tt + hf];
                    store(2 * g16, tt, i, make_float2(v[0], v[1]), make_float2(v[2], v[3]));
                }
        }
    } else {
        // accumulator register r of tile tt holds row m' = 8 (r / 4) + 4 h + r % 4 of
        // column jc: colour tt of site ts
#pragma unroll
        for (int tt = 0; tt < 3; tt++) {
            if (it >= n) continue;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                // channels a0 = 4 q + 2 h and a0 + 1: one channel pair
                const int a0 = 4 * q + 2 * h;
                if (a0 >= COUT) continue;
                store(a0, tt, it, make_float2(acc[tt][4 * q], acc[tt][4 * q + 1]),
                      make_float2(acc[tt][4 * q + 2], acc[tt][4 * q + 3]));
            }
        }
    }
}

// Weight gradient of one layer over the output sites of parity p:
//   gW[pi][a][b] += sum_{sites, colour} g_a conj(T_pi phi_b)
// Each workgroup reduces its sites through LDS; partial[blk][pi][a][b] (re, im) in FP64.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_ptc_wgrad(NetGeo g, const float2 *in, const float2 *gout, int p, long n,
                                                   double *partial)
{
    extern __shared__ unsigned char smem[];
    const int nt = blockDim.x * blockDim.y;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    cx<float> *T = (cx<float> *)smem;   // [nt][CIN*3]
    cx<float> *G = T + nt * CIN * 3;   // [nt][COUT*3]
    const int s = threadIdx.x;
    const long j = (long)blockIdx.x * blockDim.y + threadIdx.y;
    const bool valid = j < g.vh;
    const float2 *go = gout + (long)p * COUT * 3 * n;
    for (int a = 0; a < COUT; a++)
        for (int c = 0; c < 3; c++)
            G[tid * COUT * 3 + a * 3 + c] = valid ? c2(go[(a * 3 + c) * n + j * g.Ls + s]) : mk(0.f, 0.f);
    for (int pi = 0; pi < 11; pi++) {
        cx<float> t[CIN][3];
        if (valid) {
            transported<CIN>(g, in, n, p, pi, j, s, t);
        } else {
            for (int b = 0; b < CIN; b++)
                for (int c = 0; c < 3; c++) t[b][c] = mk(0.f, 0.f);
        }
        __syncthreads();
        for (int b = 0; b < CIN; b++)
            for (int c = 0; c < 3; c++) T[tid * CIN * 3 + b * 3 + c] = t[b][c];
        __syncthreads();
        for (int q = tid; q < COUT * CIN; q += nt) {
            const int a = q / CIN, b = q % CIN;
            double re = 0, im = 0;
            for (int r = 0; r < nt; r++)
                for (int c = 0; c < 3; c++) {
                    const cx<float> gg = G[r * COUT * 3 + a * 3 + c], tt = T[r * CIN * 3 + b * 3 + c];
                    // g * conj(t)
                    re += double(gg.re) * tt.re + double(gg.im) * tt.im;
                    im += double(gg.im) * tt.re - double(gg.re) * tt.im;
                }
            double *dst = partial + (((long)blockIdx.x * 11 + pi) * COUT * CIN + q) * 2;
            dst[0] = re;
            dst[1] = im;
        }
    }
}

// gw[k] (FP32, re/im interleaved) = sum over nblk partials (fixed order) [+ gw[k] when accumulate]
__global__ void k_wgrad_finish(const double *partial, int nblk, int nw, float *gw, int accumulate)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * nw) return;
    double t = 0;
    for (int b = 0; b < nblk; b++) t += partial[(long)b * 2 * nw + k];
    gw[k] = accumulate ? float(double(gw[k]) + t) : float(t);
}

// adjoint weights for the input gradient: wt[adj(pi)][b][a] = conj(w[pi][a][b])
__global__ void k_adjoint_weights(const __hip_bfloat162 *w, __hip_bfloat162 *wt, int cin, int cout)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 11 * cout * cin) return;
    const int pi = k / (cout * cin), a = (k / cin) % cout, b = k % cin;
    const int adj = (pi == 0) ? 0 : (pi <= 4) ? pi + 4 : (pi <= 8) ? pi - 4 : (pi == 9 ? 10 : 9);
    const float2 f = __bfloat1622float2(w[k]);
    wt[(adj * cin + b) * cout + a] = __float22bfloat162_rn(make_float2(f.x, -f.y));
}

// FP32 master -> BF16 working copy
__global__ void k_to_bf16(const float2 *w, __hip_bfloat162 *o, int nw)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nw) o[k] = __float22bfloat162_rn(w[k]);
}

// Adam on FP32 masters with the real-pair gradient g (= dL/dRe + i dL/dIm)
__global__ void k_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk_ = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk_;
    v[k] = vk;
    w[k] -= lr * (mk_ / c1) / (sqrtf(vk / c2) + eps);
}

// ------------------------------------------------------ spinor <-> features

// half spinor (internal layout, precision S) -> 4-channel features of parity p
// (channel = spin), the other parity zero when zero_other
template <typename S>
__global__ void __launch_bounds__(256) k_spinor_to_feat(Field f, float2 *feat, int p, long n, int zero_other)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<float> v[12];
    load_spinor<S, float>(f, i, v);
    float2 *dst = feat + (long)p * 12 * n;
    for (int c = 0; c < 12; c++) dst[c * n + i] = make_float2(v[c].re, v[c].im);
    if (zero_other) {
        float2 *o = feat + (long)(1 - p) * 12 * n;
        for (int c = 0; c < 12; c++) o[c * n + i] = make_float2(0.f, 0.f);
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_feat_to_spinor(const float2 *feat, Field f, int p, long n)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<float> v[12];
    const float2 *src = feat + (long)p * 12 * n;
    for (int c = 0; c < 12; c++) v[c] = c2(src[c * n + i]);
    store_spinor<S, float>(f, i, v);
}

// loss of one sample on parity p: r = y - x (FP32 features vs FP64 spinor x),
// partial |r|^2 and |x|^2; writes r into grad (scaled later on the host)
__global__ void __launch_bounds__(256) k_loss_residual(const float2 *y, Field x, float2 *grad, int p, long n,
                                                       double *partial)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double r2 = 0, x2 = 0;
    if (i < n) {
        cx<double> xv[12];
        load_spinor<F64, double>(x, i, xv);
        const float2 *yy = y + (long)p * 12 * n;
        float2 *gg = grad + (long)p * 12 * n;
        for (int c = 0; c < 12; c++) {
            const double dr = double(yy[c * n + i].x) - xv[c].re, di = double(yy[c * n + i].y) - xv[c].im;
            r2 += dr * dr + di * di;
            x2 += xv[c].re * xv[c].re + xv[c].im * xv[c].im;
            gg[c * n + i] = make_float2(float(dr), float(di));
        }
    }
    r2 = block_sum(r2);
    x2 = block_sum(x2);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r2;
        partial[2 * blockIdx.x + 1] = x2;
    }
}

__global__ void k_scale_feat(float2 *f, long n, float a)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) f[i] = make_float2(a * f[i].x, a * f[i].y);
}

__global__ void k_zero_feat(float2 *f, long n)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) f[i] = make_float2(0.f, 0.f);
}

// ------------------------------------------------------------ launchers

static NetGeo net_geo(Context &c)
{
    NetGeo g;
    g.nbr = c.nbr;
    g.links0 = (const float2 *)c.links_net[0];
    g.links1 = (const float2 *)c.links_net[1];
    g.nbr_sm = c.nbr_sm;
    g.lsm0 = (const float2 *)c.links[P_F32][0];
    g.lsm1 = (const float2 *)c.links[P_F32][1];
    g.vh = c.vh;
    g.Ls = c.Ls;
    return g;
}

static int net_sb(const Context &c) { return std::max(1, std::min(64, 128 / c.Ls)); }

void launch_ptc_layer(Context &c, int cin, int cout, const float2 *in, float2 *out, const void *w_bf16, int p, int pmask)
{
    const NetGeo g = net_geo(c);
    const int sb = net_sb(c);
    const dim3 grid((unsigned)((c.vh + sb - 1) / sb)), blk(c.Ls, sb);
    const __hip_bfloat162 *w = (const __hip_bfloat162 *)w_bf16;
    const double flops = (double)c.n5h * (11.0 * cout * cin * 3 * 8 + 8.0 * cin * 66);
    Timer tm(c, DWF_K_NET, (double)c.n5h * 8.0 * 3 * (11 * cin + cout), flops);
#define NETL(CI, CO) hipLaunchKernelGGL((k_ptc_fwd<CI, CO>), grid, blk, 0, c.stream, g, in, out, w, p, c.n5h, pmask)
    if (cin == 4 && cout == 12) NETL(4, 12);
    else if (cin == 12 && cout == 12) NETL(12, 12);
    else if (cin == 12 && cout == 4) NETL(12, 4);
    else if (cin == 4 && cout == 4) NETL(4, 4);
    else if (cin == 4 && cout == 8) NETL(4, 8);
    else if (cin == 8 && cout == 8) NETL(8, 8);
    else if (cin == 8 && cout == 4) NETL(8, 4);
    else if (cin == 12 && cout == 8) NETL(12, 8);
    else if (cin == 8 && cout == 12) NETL(8, 12);
    else fail(DWF_ENOTSUP, "layer channel counts must be 4, 8 or 12");
#undef NETL
    HIPCHECK(hipGetLastError());
}

// operand-order weights of the matrix-core forward: 11 cin / 4 steps x 64 lanes x 4
size_t mfma_weight_elems(int cin) { return (size_t)11 * cin / 4 * 64 * 4; }

void launch_pack_mfma_weights(Context &c, int cin, int cout, const void *w_bf16, short *pk)
{
    const __hip_bfloat162 *w = (const __hip_bfloat162 *)w_bf16;
    const dim3 grid((unsigned)((mfma_weight_elems(cin) + 255) / 256));
#define PK(CI, CO) hipLaunchKernelGGL((k_pack_mfma_weights<CI, CO>), grid, dim3(256), 0, c.stream, w, pk)
    if (cin == 4 && cout == 12) PK(4, 12);
    else if (cin == 12 && cout == 12) PK(12, 12);
    else if (cin == 12 && cout == 4) PK(12, 4);
    else if (cin == 4 && cout == 4) PK(4, 4);
    else if (cin == 4 && cout == 8) PK(4, 8);
    else if (cin == 8 && cout == 8) PK(8, 8);
    else if (cin == 8 && cout == 4) PK(8, 4);
    else if (cin == 12 && cout == 8) PK(12, 8);
    else if (cin == 8 && cout == 12) PK(8, 12);
    else fail(DWF_ENOTSUP, "layer channel counts must be 4, 8 or 12");
#undef PK
    HIPCHECK(hipGetLastError());
}

void launch_ptc_layer_mfma(Context &c, int cin, int cout, const void *in, void *out, const short *pk, int p,
                           bool in_bf16, bool out_bf16, int pmask, int io)
{
    if (((io & 1) && cin != 4) || ((io >> 1) && (out_bf16 || cout != 4 || p != 1)) || io > 5)
        fail(DWF_EINVAL, "spinor input (FP32 or BF16) or output (FP32) needs a four-channel side of the odd sites");
    const NetGeo g = net_geo(c);
    const dim3 grid((unsigned)((c.n5h + MF_S - 1) / MF_S)), blk(256);
    const double flops = (double)c.n5h * (11.0 * cout * cin * 3 * 8 + 8.0 * cin * 66);
    Timer tm(c, DWF_K_NET, (double)c.n5h * 3 * (11.0 * cin * (in_bf16 ? 4 : 8) + cout * (out_bf16 ? 4 : 8)), flops);
#define NETK(CI, CO, IB, OB) \
    hipLaunchKernelGGL((k_ptc_fwd_mfma<CI, CO, IB, OB>), grid, blk, 0, c.stream, g, in, out, pk, p, c.n5h, pmask, io)
#define NETS(CO)                                                                                               \
    hipLaunchKernelGGL((k_ptc_fwd_mfma<4, CO, true, true, true>), grid, blk, 0, c.stream, g, in, out, pk, p, \
                       c.n5h, pmask, io)
#define NETL(CI, CO)                        \
    do {                                    \
        if (in_bf16 && out_bf16)            \
            NETK(CI, CO, true, true);       \
        else if (in_bf16)                   \
            NETK(CI, CO, true, false);      \
        else if (out_bf16)                  \
            NETK(CI, CO, false, true);      \
        else                                \
            NETK(CI, CO, false, false);     \
    } while (0)
    if ((io & 1) && in_bf16) {
        // the BF16 spinor input feeds a first layer with BF16 activations out
        if (!out_bf16) fail(DWF_EINVAL, "a BF16 spinor input needs BF16 activations out");
        if (cout == 4) NETS(4);
        else if (cout == 8) NETS(8);
        else if (cout == 12) NETS(12);
        else fail(DWF_ENOTSUP, "layer channel counts must be 4, 8 or 12");
        HIPCHECK(hipGetLastError());
        return;
    }
    if (cin == 4 && cout == 12) NETL(4, 12);
    else if (cin == 12 && cout == 12) NETL(12, 12);
    else if (cin == 12 && cout == 4) NETL(12, 4);
    else if (cin == 4 && cout == 4) NETL(4, 4);
    else if (cin == 4 && cout == 8) NETL(4, 8);
    else if (cin == 8 && cout == 8) NETL(8, 8);
    else if (cin == 8 && cout == 4) NETL(8, 4);
    else if (cin == 12 && cout == 8) NETL(12, 8);
    else if (cin == 8 && cout == 12) NETL(8, 12);
    else fail(DWF_ENOTSUP, "layer channel counts must be 4, 8 or 12");
#undef NETL
#undef NETS
#undef NETK
    HIPCHECK(hipGetLastError());
}

int launch_ptc_wgrad(Context &c, int cin, int cout, const float2 *in, const float2 *gout, int p, double *partial,
                     long partial_len)
{
    const NetGeo g = net_geo(c);
    const int sb = net_sb(c);
    const long nblk = (c.vh + sb - 1) / sb;
    if (nblk * 11 * cin * cout * 2 > partial_len) fail(DWF_EINVAL, "weight-gradient buffer too small");
    const dim3 grid((unsigned)nblk), blk(c.Ls, sb);
    const size_t lds = (size_t)c.Ls * sb * (cin + cout) * 3 * sizeof(cx<float>);
    if (lds > 160 * 1024) fail(DWF_ENOTSUP, "weight-gradient tile does not fit in LDS");
    Timer tm(c, DWF_K_NET, (double)c.n5h * 8.0 * 3 * (11 * cin + cout), (double)c.n5h * 11.0 * cin * cout * 3 * 8);
#define NETW(CI, CO) hipLaunchKernelGGL((k_ptc_wgrad<CI, CO>), grid, blk, lds, c.stream, g, in, gout, p, c.n5h, partial)
    if (cin == 4 && cout == 12) NETW(4, 12);
    else if (cin == 12 && cout == 12) NETW(12, 12);
    else if (cin == 12 && cout == 4) NETW(12, 4);
    else if (cin == 4 && cout == 4) NETW(4, 4);
    else if (cin == 4 && cout == 8) NETW(4, 8);
    else if (cin == 8 && cout == 8) NETW(8, 8);
    else if (cin == 8 && cout == 4) NETW(8, 4);
    else if (cin == 12 && cout == 8) NETW(12, 8);
    else if (cin == 8 && cout == 12) NETW(8, 12);
    else fail(DWF_ENOTSUP, "layer channel counts must be 4, 8 or 12");
#undef NETW
    HIPCHECK(hipGetLastError());
    return (int)nblk;
}

void launch_wgrad_finish(Context &c, const double *partial, int nblk, int nw, float *gw, bool accumulate)
{
    hipLaunchKernelGGL(k_wgrad_finish, dim3((2 * nw + 255) / 256), dim3(256), 0, c.stream, partial, nblk, nw, gw,
                       accumulate ? 1 : 0);
    HIPCHECK(hipGetLastError());
}

void launch_adjoint_weights(Context &c, const void *w, void *wt, int cin, int cout)
{
    const int n = 11 * cin * cout;
    hipLaunchKernelGGL(k_adjoint_weights, dim3((n + 255) / 256), dim3(256), 0, c.stream, (const __hip_bfloat162 *)w,
                       (__hip_bfloat162 *)wt, cin, cout);
    HIPCHECK(hipGetLastError());
}

void launch_to_bf16(Context &c, const float *w, void *o, int nw)
{
    hipLaunchKernelGGL(k_to_bf16, dim3((nw + 255) / 256), dim3(256), 0, c.stream, (const float2 *)w,
                       (__hip_bfloat162 *)o, nw);
    HIPCHECK(hipGetLastError());
}

void launch_adam(Context &c, float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                 float eps, int step)
{
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, c.stream, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    HIPCHECK(hipGetLastError());
}

void launch_spinor_to_feat(Context &c, int prec, Field f, float2 *feat, int p, bool zero_other)
{
    const dim3 grid((unsigned)((c.n5h + 255) / 256));
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_spinor_to_feat<F64>, grid, dim3(256), 0, c.stream, f, feat, p, c.n5h, (int)zero_other); break;
    case P_F32: hipLaunchKernelGGL(k_spinor_to_feat<F32>, grid, dim3(256), 0, c.stream, f, feat, p, c.n5h, (int)zero_other); break;
    case P_F16: hipLaunchKernelGGL(k_spinor_to_feat<F16>, grid, dim3(256), 0, c.stream, f, feat, p, c.n5h, (int)zero_other); break;
    default: hipLaunchKernelGGL(k_spinor_to_feat<BF16>, grid, dim3(256), 0, c.stream, f, feat, p, c.n5h, (int)zero_other); break;
    }
    HIPCHECK(hipGetLastError());
}

void launch_feat_to_spinor(Context &c, int prec, const float2 *feat, Field f, int p)
{
    const dim3 grid((unsigned)((c.n5h + 255) / 256));
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_feat_to_spinor<F64>, grid, dim3(256), 0, c.stream, feat, f, p, c.n5h); break;
    case P_F32: hipLaunchKernelGGL(k_feat_to_spinor<F32>, grid, dim3(256), 0, c.stream, feat, f, p, c.n5h); break;
    case P_F16: hipLaunchKernelGGL(k_feat_to_spinor<F16>, grid, dim3(256), 0, c.stream, feat, f, p, c.n5h); break;
    default: hipLaunchKernelGGL(k_feat_to_spinor<BF16>, grid, dim3(256), 0, c.stream, feat, f, p, c.n5h); break;
    }
    HIPCHECK(hipGetLastError());
}

int launch_loss_residual(Context &c, const float2 *y, Field x, float2 *grad, int p)
{
    const long nb = (c.n5h + 255) / 256;
    if (2 * nb > c.partials_len) fail(DWF_EINVAL, "reduction buffer too small");
    hipLaunchKernelGGL(k_loss_residual, dim3((unsigned)nb), dim3(256), 0, c.stream, y, x, grad, p, c.n5h,
                       c.partials);
    HIPCHECK(hipGetLastError());
    return (int)nb;
}

void launch_scale_feat(Context &c, float2 *f, long n, float a)
{
    hipLaunchKernelGGL(k_scale_feat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, f, n, a);
    HIPCHECK(hipGetLastError());
}

void launch_zero_feat(Context &c, float2 *f, long n)
{
    hipLaunchKernelGGL(k_zero_feat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, f, n);
    HIPCHECK(hipGetLastError());
}

}  // namespace dwf
