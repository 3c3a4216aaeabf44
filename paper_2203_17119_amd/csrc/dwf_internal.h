// Host-side internals of the library: the context, workspaces, launch
// configuration, kernel timing and the kernel launchers implemented in the
// .hip translation units.
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/dwf.h"
#include "dwf_common.h"

namespace dwf {

// ---------------------------------------------------------------- errors

struct Error {
    dwf_status code;
    std::string msg;
};

void set_error(const std::string &m);
[[noreturn]] void fail(dwf_status code, const std::string &m);
void hip_check(hipError_t e, const char *what);
#define HIPCHECK(x) ::dwf::hip_check((x), #x)

// ------------------------------------------------------- s-local operators

// Every operator acting on the fifth dimension only is a pair of real Ls x Ls
// matrices, one for the P+ spins (0,1) and one for the P- spins (2,3).
enum SlocalOp {
    SL_A = 0,       // b + c P5
    SL_ADAG,        // b + c P5^+
    SL_MOOEE,       // d + e P5
    SL_MOOEEDAG,    // d + e P5^+
    SL_MINV,        // (d + e P5)^-1
    SL_MINVDAG,     // (d + e P5^+)^-1
    SL_E1,          // A Mee^-1           (epilogue of the first Mpc stage)
    SL_E2,          // Mee^-+ A^+         (epilogue of the first Mpc^+ stage)
    SL_AINV,        // (b + c P5)^-1      (domain-boundary projector)
    SL_NOP
};

// ------------------------------------------------------------ launch shape

struct LaunchCfg {
    int sb = 0;   // 4D sites per workgroup (workgroup = Ls x sb threads)
    int run = 1;  // XCD swizzle run length in workgroups
};

// ------------------------------------------------------------ timing

struct TimedLaunch {
    int kclass, prec;
    hipEvent_t a, b;
    double bytes, flops;
};

struct KStats {
    long launches = 0;
    double ms = 0, bytes = 0, flops = 0;
};

// ------------------------------------------------------------ context

struct Context {
    dwf_params p;
    int L[4];
    int Ls;
    long V4, vh, n5h;  // 4D sites, sites per parity, 5D sites per parity
    double d, e;       // Mooee = d + e P5
    hipStream_t stream = nullptr;
    int device = 0;
    size_t lds_max = 65536;  // dynamic LDS one workgroup may use

    int *nbr = nullptr;          // [2][8][vh] (network kernels)
    int *nbr_sm = nullptr;       // [2][vh][8], site-major (stencil)
    // Internal 4D site order, the same for both parities: internal index j of
    // the site with checkerboard index cb is perm[cb]; perm_inv[j] = cb.
    // Sites are grouped in columns of (order[0] x order[1] x order[2]) sites in
    // (x/2, y, z) that run along t, columns in lexicographic order.
    int *perm_inv = nullptr;     // device [vh]
    std::vector<int> perm_h, perm_inv_h;
    int order[3] = {0, 0, 0};
    void *links[4][2] = {};      // [prec][parity] -> [vh][8][9] elements, site-major (stencil)
    void *links_net[2] = {};     // [parity] -> FP32 [8][9][vh] (network kernels), with links[P_F32]
    double *slmat64 = nullptr;   // [SL_NOP][2][Ls][Ls]
    // operators that are twisted-circulant on one chirality block (first column
    // toep_f) and its transpose on the other; toep_rev: the P+ block is the transpose
    bool toep_ok[SL_NOP] = {};
    int toep_rev[SL_NOP] = {};
    double toep_f[SL_NOP][16] = {};
    // toep_rat: the same operator is (beta + gamma S)(delta + eps S)^-1 in the
    // twisted shift S (checked against toep_f), with |eps/delta| small enough
    // for the forward recurrence; toep_rc = {beta, gamma, delta, eps}
    bool toep_rat[SL_NOP] = {};
    double toep_rc[SL_NOP][4] = {};
    float *slmat32 = nullptr;
    double *gauge_canon = nullptr;  // canonical FP64 gauge, kept to rebuild low-precision links

    // reduction buffers
    double *partials = nullptr;  // device, nblk_max * 2
    long partials_len = 0;
    double *dscal = nullptr;     // device scalars (see solvers)
    double *hscal = nullptr;     // pinned host mirror
    // CG norm ring: coherent pinned host memory that the reduction kernel
    // writes directly (host and device addresses), one event per slot
    double *hring = nullptr, *dring = nullptr;
    hipEvent_t cg_ev[2] = {nullptr, nullptr};

    // workspaces keyed by name
    struct Buf {
        void *data = nullptr;
        float *norm = nullptr;
        size_t bytes = 0;
        int prec = -1;
        bool owned = true;  // allocated by the library (else carved from uws)
    };
    std::map<std::string, Buf> ws;
    // caller-provided workspace (dwf_set_workspace): while set, workspace
    // buffers are carved from it in order of first use, 256-byte aligned
    char *uws = nullptr;
    size_t uws_bytes = 0, uws_used = 0;

    LaunchCfg cfg_stencil, cfg_slocal, cfg_blas;
    // schedule of the batched stencil launches (several fields per launch,
    // as the multi-shift solver's), tuned apart from the single-field one
    LaunchCfg cfg_stencil_batch;

    int timing = 0;  // bit k: time launches of kernel class k
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    KStats stats[DWF_K_NCLASS];
    KStats stats_prec[DWF_K_NCLASS][4];
};

// device scalar slots and their pinned host mirror.  Slots in use: CG 0-9 and
// 250-251 (its alpha ring), FGCR 10-15, multi-shift 16 onwards (one per rhs,
// at most 64), the DD-RHMC action 246-247.
constexpr int HS_MIRROR = 256;

// default 4D sites per workgroup: about 192 lanes
// 4D sites per workgroup by default: about 192 lanes, at most 64 sites
inline int default_sb(const Context &c) { return c.Ls >= 192 ? 1 : std::min(64, 192 / c.Ls); }
inline int cfg_sb(const Context &c, const LaunchCfg &g) { return g.sb > 0 ? g.sb : default_sb(c); }

// sizes
size_t elem_bytes(int prec);
size_t field_bytes(const Context &c, long n5, int prec);

// workspace field of one parity in precision prec (allocated on first use)
Field ws_field(Context &c, const std::string &name, int prec);
// untyped workspace buffer of at least `bytes` (allocated on first use)
void *ws_raw(Context &c, const std::string &name, size_t bytes);

// One workspace buffer an operation takes: a field (nbatch == 0: one field by
// ws_field; nbatch >= 1: a batch by ws_batch) or raw bytes (prec < 0).
struct WsKey {
    std::string name;
    int prec;
    int nbatch;
    size_t raw;
};
// bytes the buffers of a plan take in a caller workspace (each 256-aligned)
size_t ws_plan_bytes(const Context &c, const std::vector<WsKey> &plan);
Field make_field(const Context &c, void *data, int prec);  // caller memory (FP16: norm follows data)

const void *slmat(const Context &c, int op, bool f64);

// timing helpers
struct Timer {
    Context &c;
    int kclass, prec;
    double bytes, flops;
    hipEvent_t a = nullptr;
    // prec: storage precision of the launch's fields, -1 when not specific
    Timer(Context &c_, int k, double by, double fl, int pr = -1);
    ~Timer();
};

// --------------------------------------------------------- kernel launchers

// choose the column cross-section (in x/2, y, z) of the internal site order;
// zeros pick the default for the lattice size
void build_order(Context &c, int cxh, int cy, int cz);
long column_sites(const Context &c);
void ensure_links(Context &c, int prec);
void default_schedule(Context &c);
// build the neighbour table on the host and upload; prepare links in prec
void build_neighbours(Context &c);
void prepare_links(Context &c, int prec);

// canonical FP64 <-> internal (one parity); full canonical fields are read at
// the sites of parity `parity` when full != 0
void launch_import(Context &c, int prec, const double *canon, Field out, int full, int parity);
void launch_export(Context &c, int prec, Field in, double *canon, int full, int parity);
void launch_convert(Context &c, int pin, Field in, int pout, Field out);

// Fused stencil: out = sigma * Self(self) + tau * Epi(H_{p,1-p} in)
struct StencilSpec {
    int out_parity = 0;
    bool dagger = false;
    int epi = EPI_NONE;
    int epi_op = -1;          // SlocalOp for EPI_DENSE
    double e0 = 0, e1 = 0;    // EPI_SHIFT: e0 + e1 P5 (edag: P5^+)
    bool edag = false;
    bool self = false;        // add sigma * (s0 + s1 P5) self
    double s0 = 0, s1 = 0;
    bool sdag = false;
    double sigma = 1.0, tau = 1.0;
    bool reduce = false;      // per-workgroup |out|^2 partials into c.partials
    bool cg_update = false;   // out = out - dscal[alpha_slot] * result (needs reduce)
    int alpha_slot = -1;
    int kclass = DWF_K_STENCIL;
    int nbatch = 1;           // fields processed in one launch (blockIdx.y), member k of
    long bstride = 0;         // in/self/out at data + k*bstride bytes; partials [k][block]
};
// prec: storage precision of in/out/self; FP64 uses double arithmetic, the
// others float.  Returns the number of partials written when reduce is set.
int launch_stencil(Context &c, int prec, const StencilSpec &sp, Field in, Field self, Field out);

// domain boundary (two-flavour boundary action): mask[n] over the lexicographic
// 4D sites, nonzero on the domain.  Links between the domains zeroed (canonical
// FP64 gauge fields, gin and gout may alias); on one parity of an FP64 field,
// kind 0 applies the spin-space mask of the boundary sites, kind 1 keeps the
// field on the domain (in and out may alias).
void launch_mask_links(Context &c, const int8_t *mask, const double *gin, double *gout);
void launch_boundary_mask(Context &c, const int8_t *mask, Field in, Field out, int parity, int kind);

// s-local operator e0 + e1 P5 (dag: P5^+) from the fifth-dimension neighbours
// (A, A^+, Mooee, Mooee^+; launch_slocal uses it for those); in and out may alias
void launch_slocal_shift(Context &c, int prec, double e0, double e1, bool dag, Field in, Field out, int nbatch = 1,
                         long bstride = 0);

// s-local dense operator out = M in (M one of SlocalOp); in and out may alias
void launch_slocal(Context &c, int prec, int op, Field in, Field out, int nbatch = 1, long bstride = 0);

// batches of fields: member k of a batch starting at field f lies k*batch_stride
// bytes after it (field bytes rounded up to 256)
long batch_stride(const Context &c, int prec);
Field ws_batch(Context &c, const std::string &name, int prec, int nbatch);
__host__ __device__ inline Field member(Field f, int k, long stride)
{
    f.data = (char *)f.data + (long)k * stride;
    if (f.norm) f.norm = (float *)((char *)f.norm + (long)k * stride);
    return f;
}

// device state of the batched multi-shift solver
struct MsState {
    double *rho, *pap, *alpha, *alpha_old, *beta_old, *target;  // [nrhs]
    double *zeta, *zeta_old;                                      // [nshift*nrhs]
    int *active, *iters;                                          // [nshift*nrhs]
    double *coef;                                                 // [nshift*nrhs][4] (a, z, b, on)
    double *shifts;                                               // [nshift]
};
void ms_launch_norm2(Context &c, int prec, Field a, int nb, long stride, double *out);
// out[j] = Re<a_j, b_j> + sigma |a_j|^2
void ms_launch_redot(Context &c, int prec, Field a, Field b, int nb, long stride, double *out, double sigma = 0.0);
// One multi-shift step: alpha, r -= alpha (ap + sigma pbase) (ap: the normal
// operator applied to the carrier's directions pbase, sigma: the carrier's
// shift), |r|^2, the shift recurrences (coefficients into s.coef), then the
// shifted directions into Pn and the operator's first factor of the carrier's
// new directions into ta.  Solution updates go in pairs (see k_ms_update_b):
// an odd it leaves its update pending (direction in P, coefficients in
// s.coef), the next applies it from Pn with the coefficients cprev, and its own.
void ms_launch_step(Context &c, int prec, const MsState &s, Field r, Field ap, Field X, Field P, Field Pn,
                    const double *cprev, int nrhs, int nshift, int kmin, long stride, double *rho_new, int it,
                    Field pbase, double sigma, Field ta);
// x += a p for every member whose coefficients in coef are on
void ms_launch_flush(Context &c, int prec, Field X, Field P, const double *coef, int nrhs, int nshift, long stride);

// reductions: partial sums (2 doubles per workgroup for dots) then a fixed-order
// finish on the device that writes dscal[slot] (and dscal[slot+1] for dots)
int launch_norm2(Context &c, int prec, Field a);
int launch_dot(Context &c, int prec, Field a, Field b);
// dscal[slot + w] = sum of the partials; mirror (device-visible host memory),
// when given, receives the same values; with qslot >= 0 (width 1) also
// dscal[qslot] = dscal[nslot] / sum
void launch_finish(Context &c, int nparts, int width, int slot, double *mirror = nullptr, int qslot = -1,
                   int nslot = -1);
// dscal[slot] = v, queued on the stream (the host does not wait)
void launch_set_scalar(Context &c, int slot, double v);
// dscal[beta] = dscal[rho_new] / dscal[rho], then dscal[rho] = dscal[rho_new]
void launch_cg_beta(Context &c, int beta, int rho, int rho_new);

// generic vector ops with host scalars: z = a*x + b*y (real a, b)
void launch_axpby(Context &c, int prec, double a, Field x, double b, Field y, Field z);
// z = a x + b y + cc w
void launch_axpbypcz(Context &c, int prec, double a, Field x, double b, Field y, double cc, Field w, Field z);
// complex caxpy with host scalar: y += a * x
void launch_caxpy(Context &c, int prec, double are, double aim, Field x, Field y);
void launch_zero(Context &c, int prec, Field a);
void launch_copy(Context &c, int prec, Field a, Field b);

// precision of the low-precision solution accumulator for a sloppy precision
inline int accum_prec(int prec) { return (prec == P_F16 || prec == P_BF16) ? P_F32 : prec; }

// CG building blocks with device scalars
// x += alpha p ; r -= alpha ap ; partials of |r|^2        (alpha = dscal[ia];
// x in accum_prec(prec), the others in prec)
int launch_cg_update_xr(Context &c, int prec, Field x, Field r, Field p, Field ap, int ia);
// Older CG directions whose solution updates are still pending, oldest first,
// with the device slots of their alphas.
struct CgOlder {
    static constexpr int MAX = 3;
    Field dir[MAX];
    int slot[MAX] = {-1, -1, -1};
    int n = 0;
};
// pout = r + beta p, pa = A pout (A = b + c P5, beta = dscal[ib]).  With ia >= 0
// the pending solution updates come first: x += alpha_j q_j over `older`, then
// x += alpha p (alpha = dscal[ia]; x in the accumulator precision of prec).
// pout may alias p or one of the older directions.
void launch_cg_update_p(Context &c, int prec, Field r, Field p, Field pout, Field pa, int ib, Field x = Field{},
                        int ia = -1, const CgOlder &older = CgOlder{});
// Block Gram-Schmidt of flexible GCR (FP64 or FP32 fields as flat complex
// arrays, FP64 sums).  gs_dots: out[2j], out[2j+1] = Re, Im <X_j, y>, j < nv
// (X_dev: device array of nv field pointers; partial: gs_partials_needed
// doubles).  gs_project: y -= sum b_j X_j, w -= sum b_j W_j, b_j = <X_j, y> /
// nq[3 j]; out = {|y|^2, Re <y, r>, Im <y, r>}.  gs_update: x += a z, r -= a q
// with a = (coef[1] + i coef[2]) / coef[0]; returns the number of |r|^2
// partials written to c.partials.
long gs_partials_needed(const Context &c, int nv);
void launch_gs_dots(Context &c, int prec, const void *const *X_dev, int nv, Field y, double *partial, double *out);
// prec is the precision of the basis vectors (X, W, y, w, z, q), rprec that of
// the residual r and the solution x: FP64/FP64, FP32/FP32 or BF16/FP32.  With
// an empty w (and no W_dev; BF16 basis only) y alone is projected.
void launch_gs_project(Context &c, int prec, int rprec, const void *const *X_dev, const void *const *W_dev, int nv,
                       const double *dots, const double *nq, Field y, Field w, Field r, double *partial, double *out);
// rb (BF16 basis only): also write the updated r rounded to BF16
int launch_gs_update(Context &c, int prec, int rprec, Field x, Field z, Field r, Field q, const double *coef,
                     Field rb = {});
// BF16 basis: x += sum_j a_j Z_j over nz directions (Z_dev: device array of
// their pointers), a_j from coef[3j..3j+2] as in gs_update; x FP32.  With it
// the per-step update may pass an empty x.
void launch_gs_combine(Context &c, int prec, Field x, const void *const *Z_dev, int nz, const double *coef);
// coefficients cc (3 nz doubles, the form gs_combine reads) that combine nz
// unprojected directions into the update the projected ones would give:
// dots[k stride ..] holds step k's projection dots, nq the per-step info
// {|q_k|^2, <q_k, r>}; one thread on the device
void launch_gs_raw_coef(Context &c, int nz, int stride, const double *dots, const double *nq, double *cc);
// x += dscal[ia] p, x in the accumulator precision of prec
void launch_axpy_dev(Context &c, int prec, Field x, Field p, int ia);
// device scalar arithmetic: dscal[out] = dscal[num] / dscal[den]
void launch_scalar_div(Context &c, int out, int num, int den);
// r_h = b - ax (FP64), partials of |r_h|^2
int launch_residual(Context &c, Field b, Field ax, Field r);
// xh += xl (FP64 += prec), xl = 0
void launch_accumulate_low(Context &c, int prec, Field xh, Field xl);
// multi-shift: for shifts k with coef[k] active: x_k += a_k p_k ; p_k = z_k r + b_k p_k
void launch_ms_update(Context &c, int prec, int nshift, Field *x, Field *p, Field r, const double *coef_dev,
                      const int *active_host);

// resolve the device address of the fixed scratch array on `device` (the
// current device); called once per context creation
void scratch_init(int device);

void read_scalars(Context &c, int first, int count);  // dscal -> hscal, synchronising
void launch_stream_copy(Context &c, const void *src, void *dst, size_t bytes);
// bandwidth probes (kind 0 copy, 1 read-only, 2 two reads per write), unroll
// loads in flight per lane (1, 2, 4 or 8), non-temporal when nt
long stream_probe_blocks(size_t bytes, int unroll);
void launch_stream_probe(Context &c, int kind, int unroll, bool nt, const void *a, const void *b, void *dst,
                         size_t bytes);

// ---------------------------------------------------------------- Mpc helpers

// out = Mpc in (dagger: Mpc^+) in precision prec, using workspaces of that
// precision; if reduce, partials of |out|^2 are written and their count returned.
// With dagger and alpha_slot >= 0 the result is not stored: out holds a
// residual r on entry and becomes r - dscal[alpha_slot] Mpc^+ in, with the
// partials of its |r|^2 (reduce implied).  The intermediate fields are
// context workspaces unless ws_ta and ws_y are given (one field each, or with
// nbatch > 1 batches of at least nbatch members at the batch stride); ws_ta
// is needed only when in_is_A_applied is false and dagger is not set.
int apply_mpc(Context &c, int prec, bool dagger, Field in, Field out, bool reduce, bool in_is_A_applied = false,
              Field pa = Field{}, int nbatch = 1, long bstride = 0, int alpha_slot = -1, Field ws_ta = Field{},
              Field ws_y = Field{});

}  // namespace dwf

// the opaque handle of the C ABI
struct dwf_context : public dwf::Context {};

// Body of every C entry point: errors thrown inside become a status and the
// thread-local message; falling through the body returns DWF_OK.
#define DWF_API_BEGIN try {
#define DWF_API_END                              \
    return DWF_OK;                               \
    }                                            \
    catch (const dwf::Error &e)                  \
    {                                            \
        dwf::set_error(e.msg);                   \
        return e.code;                           \
    }                                            \
    catch (const std::exception &e)              \
    {                                            \
        dwf::set_error(e.what());                \
        return DWF_ENOMEM;                       \
    }
