/*
 * dwf.h -- C ABI of the MI355X (gfx950) domain-wall fermion library.
 *
 * The library applies the red-black preconditioned Moebius domain-wall Dirac
 * operator and solves with it on one GPU's block of the lattice, the local
 * Dirichlet solves of domain-decomposed HMC (Boyle, Bollweg, Kelly,
 * Yamaguchi, "Algorithms for Domain Wall Fermions", Sec. 2.3 and 2.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns a dwf_status; DWF_OK on success.  On error
 *   nothing is launched (argument errors) or the device error is reported
 *   (DWF_EDEVICE); dwf_last_error() returns a thread-local message.
 * Memory: the caller owns every field buffer and passes raw pointers; unless
 *   stated otherwise they are DEVICE pointers on the context's device.  The
 *   library owns its context, the internal gauge copies and its workspaces and
 *   frees them in dwf_destroy.  No call keeps a caller pointer after it returns.
 * Streams: work is enqueued on the context's hipStream_t (set at create time or
 *   by dwf_set_stream).  Operator calls are asynchronous; solver calls
 *   synchronise the stream before they return their statistics.
 * Lattice: extents L = (Lx, Ly, Lz, Lt), each even and >= 2, fifth dimension
 *   Ls >= 1.  Site n = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t) mod 2,
 *   checkerboard index cb = n >> 1.  Boundary conditions are periodic unless
 *   the face is Dirichlet.
 * Canonical layouts (complex numbers as interleaved (re, im) doubles):
 *   gauge        [n][mu = x,y,z,t][row 3][col 3], U_mu(x) is the link x -> x+mu
 *   full fermion [n][s][spin 4][colour 3]
 *   half fermion [cb][s][spin 4][colour 3], the sites of one parity
 * Gamma matrices (chiral basis): gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 *   for k = x,y,z, gamma_t = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 * Operator (the paper's DWF action objects; written out following Brower,
 * Neff and Orginos since the paper does not print it):
 *   H psi(x)  = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
 *   D_W       = (4 - M5) - H/2
 *   P5 psi_s  = P_- psi_{s+1} + P_+ psi_{s-1}, psi_Ls = -mf psi_0, psi_-1 = -mf psi_{Ls-1}
 *   D5        = (b D_W + 1) + (c D_W - 1) P5 = Mooee - H A / 2
 *   A = b + c P5, Mooee = d + e P5, d = b(4-M5)+1, e = c(4-M5)-1
 *   Mpc       = Mooee - (1/4) H_oe A Mooee^-1 H_eo A   on odd sites
 * Internal layouts are private; dwf_import/dwf_export convert to and from them
 * for callers that keep fields in the library's own layout and precision.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dwf_status;
enum {
    DWF_OK = 0,
    DWF_EINVAL = -1,   /* bad dimensions, parameters or null pointer            */
    DWF_ENOMEM = -2,   /* device or host allocation failed                      */
    DWF_EDEVICE = -3,  /* a HIP call failed                                     */
    DWF_ENOCONV = -4,  /* solver reached maxit or stagnated; outputs hold the
                          last iterate and the statistics are filled            */
    DWF_ENOTSUP = -5   /* precision or option not supported                     */
};

/* storage precisions of internal fields */
enum {
    DWF_F64 = 0,   /* double complex                                         */
    DWF_F32 = 1,   /* float complex                                          */
    DWF_F16 = 2,   /* half complex, one float scale per 5D site (spinors)    */
    DWF_BF16 = 3   /* bfloat16 complex                                       */
};

typedef struct dwf_context *dwf_ctx;

typedef struct {
    int dims[4];       /* local lattice extents, each even and >= 2              */
    int Ls;            /* extent of the fifth dimension, >= 1                    */
    double b, c;       /* Moebius coefficients (Shamir: b = 1, c = 0)            */
    double M5;         /* domain-wall height                                     */
    double mf;         /* quark mass                                             */
    int dirichlet[4];  /* 1: zero the links leaving the block through the face
                          x_mu = L_mu - 1 (Sec. 2.4: Dirichlet boundary
                          conditions applied to the gauge-field argument)      */
} dwf_params;

int dwf_abi_version(void);
const char *dwf_last_error(void);

/* Create a context on the current HIP device.  gauge: canonical FP64 field,
 * a device pointer when gauge_on_device != 0, else host memory.  The links
 * crossing each flagged Dirichlet face are zeroed in the internal copies
 * (Sec. 2.4).  stream: a hipStream_t (NULL = default stream). */
dwf_status dwf_create(const dwf_params *p, const double *gauge, int gauge_on_device, void *stream,
                      dwf_ctx *out);
dwf_status dwf_destroy(dwf_ctx ctx);
/* Replace the gauge field (same geometry and parameters). */
dwf_status dwf_set_gauge(dwf_ctx ctx, const double *gauge, int on_device);
dwf_status dwf_set_stream(dwf_ctx ctx, void *stream);

/* ------------------------------------------------------------ workspaces
 *
 * The library's workspace fields (solver vectors, the operators'
 * intermediates) are allocated on first use and kept by the context, unless
 * the caller hands it a device buffer: while one is set, every workspace
 * buffer is carved from it (256-byte aligned, in order of first use), so that
 * the caller's allocator owns that memory.  The context's own state (the
 * gauge copies per precision, neighbour tables, reduction scalars) stays
 * library-owned: dwf_create allocates it, and the links of a storage precision
 * other than FP64 on first use or by dwf_prepare_links. */
enum {
    DWF_OP_CG = 0,           /* dwf_cg in `mode`                                       */
    DWF_OP_MULTISHIFT = 1,   /* dwf_multishift_cg in `mode` with nrhs x nshift systems */
    DWF_OP_RATIONAL = 2,     /* dwf_rational_apply, `nshift` poles (nrhs ignored)      */
    DWF_OP_SCHUR_APPLY = 3,  /* dwf_schur_apply (mode, nrhs, nshift ignored)           */
    DWF_OP_BOUNDARY = 4      /* dwf_boundary_apply on the full context, solves in
                                `mode` (nrhs, nshift ignored; the cut context's own
                                solves need DWF_OP_CG there)                       */
};
/* Bytes of caller workspace the operation needs on a context that has none
 * of its buffers yet (an upper bound otherwise).  DWF_EINVAL for an unknown
 * op or sizes out of range, DWF_ENOTSUP for a mode the operation lacks. */
dwf_status dwf_workspace_bytes(dwf_ctx ctx, int op, int mode, int nrhs, int nshift, size_t *bytes);
/* Hand the context a device buffer (256-byte aligned; NULL returns to library
 * allocation).  Buffers carved from an earlier caller workspace are forgotten
 * (the caller may free it after this call); the library's own earlier
 * allocations stay.  A later call that needs more than is left returns
 * DWF_ENOMEM and names the size.  The buffer must stay valid while set. */
dwf_status dwf_set_workspace(dwf_ctx ctx, void *ws, size_t bytes);
/* Bytes of the caller workspace in use (0 when none is set). */
dwf_status dwf_workspace_used(dwf_ctx ctx, size_t *bytes);
/* Prepare the links in storage precision prec now (they are otherwise
 * prepared by the first call in that precision). */
dwf_status dwf_prepare_links(dwf_ctx ctx, int prec);

/* Bytes of one internal field: full != 0 for both parities, else one parity. */
dwf_status dwf_field_bytes(dwf_ctx ctx, int full, int prec, size_t *bytes);
/* Convert a canonical FP64 half field (full == 0) to the internal layout in
 * precision prec, and back.  Device pointers. */
dwf_status dwf_import(dwf_ctx ctx, int full, int prec, const double *canon, void *internal);
dwf_status dwf_export(dwf_ctx ctx, int full, int prec, const void *internal, double *canon);

/* Raw Wilson hop on every s slice, from parity 1-out_parity to out_parity:
 * out = H in (dagger = 0) or H^+ in = g5 H g5 in (dagger = 1).  No -1/2 and no
 * A factor.  Canonical FP64 half fields. */
dwf_status dwf_dhop(dwf_ctx ctx, int out_parity, int dagger, const double *in_half, double *out_half);
/* Same operator on internal half fields of precision prec (FP64 math for
 * DWF_F64, FP32 math otherwise). */
dwf_status dwf_dhop_internal(dwf_ctx ctx, int prec, int out_parity, int dagger, const void *in, void *out);

/* s-local diagonal block Mooee = d + e P5 (dagger: d + e P5^+) and its inverse,
 * applied on a canonical FP64 half field of either parity. */
dwf_status dwf_mooee(dwf_ctx ctx, int dagger, const double *in_half, double *out_half);
dwf_status dwf_mooeeinv(dwf_ctx ctx, int dagger, const double *in_half, double *out_half);

/* Odd-site Schur complement Mpc (dagger = 0) or Mpc^+ (dagger = 1) of the
 * red-black decomposition; canonical FP64 odd half fields. */
dwf_status dwf_schur_apply(dwf_ctx ctx, int dagger, const double *in_odd, double *out_odd);
/* Same on internal odd fields of precision prec; in and out must differ. */
dwf_status dwf_schur_apply_internal(dwf_ctx ctx, int prec, int dagger, const void *in, void *out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same operator
 * and the same kernels as dwf_schur_apply_internal, with the intermediate
 * fields in a fixed device array of 128 MiB per device instead of context
 * workspaces, and no allocation of any kind (kernel timing is off for the
 * call).  The array holds two intermediate fields of precision prec (one for
 * dagger = 1): DWF_EINVAL when batch-aligned field bytes exceed that (e.g.
 * FP64 beyond about 350k odd 5D sites).  The links of prec must already be
 * prepared (FP64 always is; other precisions after any earlier operator or
 * solver call in that precision), else DWF_EINVAL.  Every call on one device
 * shares the array: calls that overlap on one device (different streams or
 * host threads) race and must be serialised by the caller; nothing in the
 * array needs to start at zero. */
dwf_status dwf_schur_apply_internal_noalloc(dwf_ctx ctx, int prec, int dagger, const void *in, void *out);

/* --------------------------------------------------------------- solvers */

enum {
    DWF_SOLVE_F64 = 0,        /* FP64 storage and arithmetic                        */
    DWF_SOLVE_MIXED_F32 = 1,  /* FP32 storage and arithmetic, FP64 reliable updates */
    DWF_SOLVE_MIXED_F16 = 2,  /* FP16 storage (+ per-site scale), FP32 arithmetic   */
    DWF_SOLVE_MIXED_BF16 = 3  /* BF16 storage, FP32 arithmetic                      */
};

typedef struct {
    double tol;        /* stop when |r| <= tol |rhs| (normal equations for CG)    */
    int maxit;         /* iteration limit (<= 0: 100000)                          */
    int mode;          /* DWF_SOLVE_*                                             */
    double delta;      /* reliable-update threshold (<= 0: 0.1): the FP64 residual
                          is recomputed once the iterated one has fallen by this
                          factor, and after 150 iterations without an update.
                          Larger values recompute more often; with FP16 storage
                          on an ill-conditioned operator that saves iterations
                          (see the design notes on 24^4 x 12)                   */
    int x0_is_guess;   /* 1: x holds an initial guess on entry                    */
    int restart;       /* FGCR restart length m (<= 0: 16)                         */
    int normal;        /* FGCR: 1 solves the normal equations Mpc^+ Mpc, 0 Mpc    */
    int fallback;      /* FGCR: 1 falls back to CG on stagnation / NaN            */
    int tile_sb;       /* multi-shift: schedule of its batched stencil launches:
                          0 keeps the context's DWF_SCHED_STENCIL_BATCHED schedule,
                          > 0 sets it to 4D sites per workgroup (with tile_run),
                          -1 autotunes it (dwf_tune_op, no cache); a schedule set
                          or tuned here stays set on the context */
    int tile_run;      /* multi-shift with tile_sb > 0: XCD run length (>= 1)     */
} dwf_solver_opts;

typedef struct {
    int iters;              /* Krylov iterations                                   */
    int reliable_updates;   /* FP64 residual recomputations (mixed precision)      */
    int converged;          /* 1 when the FP64 residual met tol                    */
    int fell_back;          /* FGCR: 1 when the CG fallback produced the answer    */
    double res_normal;      /* |Mpc^+(b~ - Mpc x)| / |Mpc^+ b~|                    */
    double res_schur;       /* |b~ - Mpc x| / |b~|                                 */
    double res_full;        /* |b - D5 x| / |b| (full solves only)                 */
    double seconds;         /* wall time of the call                               */
    double t_prep, t_solve, t_final; /* source preparation, Krylov loop, reconstruction
                                        plus FP64 residual check                    */
} dwf_solver_stats;

/* Solve D5 x = b: Schur source b~_o = b_o - Moe Mee^-1 b_e, CG on
 * Mpc^+ Mpc x_o = Mpc^+ b~_o, x_e = Mee^-1 (b_e - Meo x_o) (the "usual red-black
 * preconditioned" local solve, Sec. 2.3).  Canonical FP64 full fields. */
dwf_status dwf_cg(dwf_ctx ctx, const double *b_full, double *x_full, const dwf_solver_opts *o,
                  dwf_solver_stats *st);

/* Multi-shift CG: (Mpc^+ Mpc + shifts[k]) x[j*nshift + k] = b[j] for every
 * right-hand side j < nrhs and shift k < nshift, one Krylov space per j (the
 * rational-function solves of the DD-RHMC one-flavour action, Sec. 2.3.1).
 * b and x are arrays of canonical FP64 odd half fields (device pointers, the
 * pointer arrays themselves in host memory); st has nrhs*nshift entries (may
 * be NULL).  mode DWF_SOLVE_F64 or DWF_SOLVE_MIXED_F32 (FP32 Krylov space).
 * Every solution's residual is then recomputed in FP64.  In MIXED_F32 the
 * systems that miss the tolerance are refined by defect correction: the FP64
 * residuals of the right-hand sides of one shift are solved together, in FP32
 * storage, and the corrections kept in a second FP32 term beside the solution
 * (up to four passes, then the single-system mixed CG).  st[].reliable_updates
 * counts a system's refinement iterations. */
dwf_status dwf_multishift_cg(dwf_ctx ctx, int nrhs, const double *const *b_odd, int nshift,
                             const double *shifts, double *const *x_odd, const dwf_solver_opts *o,
                             dwf_solver_stats *st);

/* ------------------------------------------------------------- DD-RHMC */

/* A rational function in partial fractions,
 *   r(x) = a0 + sum_{k < n} alpha[k] / (x + beta[k]),   1 <= n <= 64, beta[k] >= 0,
 * the form in which the one-flavour (RHMC) actions apply fractional powers of
 * a normal operator.  alpha and beta are host arrays.  The library evaluates
 * r; the coefficients (e.g. a best relative approximation of x^p on an interval
 * covering the spectrum, computed by paper_2203_17119_amd/rational/remez.py)
 * are the caller's. */
typedef struct {
    int n;
    double a0;
    const double *alpha;
    const double *beta;
} dwf_rational;

/* out = r(A) in with A = Mpc^+ Mpc of the context: one multi-shift solve with
 * the shifts beta[k] (modes and tolerance of dwf_multishift_cg: every shifted
 * system meets o->tol in FP64), then out = a0 in + sum_k alpha[k] x_k on the
 * device.  in_odd and out_odd are canonical FP64 odd half fields (device; they
 * may be the same buffer).  st (may be NULL) receives the statistics of the
 * worst shifted system (largest iteration count, converged only when all are).
 * Errors: DWF_EINVAL for a null pointer, n outside 1..64, negative or
 * non-finite beta, non-finite a0 or alpha; DWF_ENOCONV when a shift missed the
 * tolerance (out then holds the combination of the last iterates). */
dwf_status dwf_rational_apply(dwf_ctx ctx, const dwf_rational *r, const double *in_odd, double *out_odd,
                              const dwf_solver_opts *o, dwf_solver_stats *st);

/* The one-flavour boundary action of DD-RHMC (Sec. 2.3.1, following eq.
 * (ddrhmc)): with A = Mpc^+ Mpc of ctx (the operator of the whole lattice) and
 * A_d that of ctx_dirichlet (the same field with its Dirichlet faces cut),
 *   S = phi^+ r_q(A_d) r_m(A) r_q(A_d) phi,   r_q ~ x^{1/4},  r_m ~ x^{-1/2},
 * evaluated as psi = r_q(A_d) phi, chi = r_m(A) psi, S = Re <psi, chi> (FP64
 * sum on the device).  Since det D5 = det Mee det Mpc with Mee field-independent,
 * a Gaussian phi with this action samples det D / det D_dirichlet, the
 * boundary determinant of eq. (ddrhmc).  The two contexts must have the same
 * lattice, Ls and operator parameters.  phi_odd: canonical FP64 odd half field
 * (device).  action: host.  st (may be NULL): two entries, the r_q and r_m
 * solves as in dwf_rational_apply.  Errors as dwf_rational_apply, and
 * DWF_EINVAL for contexts of different geometry or parameters. */
dwf_status dwf_ddrhmc_action(dwf_ctx ctx, dwf_ctx ctx_dirichlet, const dwf_rational *r_quarter,
                             const dwf_rational *r_minus_half, const double *phi_odd, const dwf_solver_opts *o,
                             double *action, dwf_solver_stats *st);

/* Chebyshev filter of the normal operator A = Mpc^+ Mpc: the recursively
 * generated filter functions proposed for fast multigrid subspace set-up of
 * the local Dirichlet solves (Sec. 2.4 and its filter-function figure).  With
 * x(A) = (2 A - (hi + lo)) / (hi - lo) mapping [lo, hi] onto [-1, 1],
 *   w_0 = v,  w_1 = x(A) v,  w_{k+1} = 2 x(A) w_k - w_{k-1},
 * so w_k = T_k(x(A)) v: eigencomponents of A inside [lo, hi] are bounded by
 * |T_k| <= 1, those below lo grow like cosh(k acosh |x|).  out_odd[i] receives
 * w_{orders[i]} for nout (1..64) strictly ascending orders in [0, 100000].
 * prec (DWF_F64/F32/F16/BF16) is the storage precision of the recurrence
 * (FP64 arithmetic for DWF_F64, FP32 otherwise).  v_odd and the out_odd[i]
 * are canonical FP64 odd half fields (device); orders and the out_odd array
 * live in host memory.  The call returns when the work is queued on the
 * context's stream; it uses context workspace (five fields of prec).
 * Errors: DWF_EINVAL for a null pointer, unknown prec, nout outside 1..64,
 * orders not ascending or out of range, or unless 0 <= lo < hi (finite). */
dwf_status dwf_chebyshev_filter(dwf_ctx ctx, int prec, const double *v_odd, double lo, double hi, int nout,
                                const int *orders, double *const *out_odd);

/* ------------------------------------------------------ domain boundary */

/* The two-flavour boundary action (Sec. 2.1, the construction after eq.
 * (schur)) splits the lattice into a domain Omega and its complement
 * Omega-bar.  mask (device, int8, one entry per lexicographic 4D site
 * n = x + Lx (y + Ly (z + Lz t))) is 1 on Omega and 0 on Omega-bar; every
 * entry must be 0 or 1 and both domains non-empty (else DWF_EINVAL).  The
 * boundary is found by comparing the mask with its shift by one site in each
 * direction (Sec. 2.4, "Results"). */

/* gauge_out = gauge_in with every link U_mu(x) whose ends x, x + mu lie in
 * different domains set to zero (canonical FP64 gauge fields [n][mu][3][3],
 * device; they may be the same buffer; the context supplies the lattice and
 * stream).  A context created from the result applies the block-diagonal
 * operator D_cut = diag(D_Omega, D_Omegabar) of eq. (schur). */
dwf_status dwf_mask_links(dwf_ctx ctx, const int8_t *mask, const double *gauge_in, double *gauge_out);

/* out = D5 in on canonical FP64 full fields (device). */
dwf_status dwf_d5_apply(dwf_ctx ctx, const double *in_full, double *out_full);

/* out = P in: the projector onto the components of a field on Omega that the
 * boundary block D_dbar (Omega to Omega-bar) acts on, D_dbar P = D_dbar.  With
 * D5 = Mooee - (1/2) H A the boundary hop sees (1 + gamma_mu) A psi at a site
 * of Omega whose neighbour x + mu is in Omega-bar and (1 - gamma_mu) A psi for
 * x - mu, so P = A^-1 Pi A, Pi being (1 +- gamma_mu)/2 at a boundary site with
 * one neighbour in Omega-bar, 1 with two or more (the two ranges span all
 * spins), 0 elsewhere (oblique for c != 0; for Shamir the orthogonal spin
 * mask).  Canonical FP64 full fields (device).  DWF_ENOTSUP when
 * A = b + c P5 is singular (b = 0). */
dwf_status dwf_boundary_project(dwf_ctx ctx, const int8_t *mask, const double *in_full, double *out_full);

/* out = R psi (inverse = 0) or R^-1 psi (inverse = 1) for the part of psi on
 * Omega, with
 *   R    = P - P D_Omega^-1 D_d D_Omegabar^-1 D_dbar,
 *   R^-1 = P - P D^-1 D_dbar,
 * D the operator of ctx and D_cut = diag(D_Omega, D_Omegabar) that of ctx_cut
 * (the same lattice and parameters, its gauge field cut by dwf_mask_links with
 * the same mask), D_d + D_dbar = D - D_cut.  R R^-1 = P, and det R on the
 * range of P is the boundary determinant det(1 - D_Omega^-1 D_d D_Omegabar^-1
 * D_dbar).  R takes two solves with ctx_cut, R^-1 one with ctx (dwf_cg with
 * o, its x0_is_guess ignored).  Canonical FP64 full fields (device).  st (may
 * be NULL): iterations and reliable updates summed over the solves, the
 * largest of their residuals, converged when all are, wall time in seconds.
 * Errors: DWF_EINVAL for null pointers, ctx_cut == ctx, contexts of different
 * lattice or parameters, a bad mask or inverse; DWF_ENOCONV when a solve
 * missed the tolerance (out is then computed from its last iterate). */
dwf_status dwf_boundary_apply(dwf_ctx ctx, dwf_ctx ctx_cut, const int8_t *mask, int inverse, const double *in_full,
                              double *out_full, const dwf_solver_opts *o, dwf_solver_stats *st);

/* ---------------------------------------------- learned preconditioner */

/* A gauge-equivariant network of parallel-transport convolution layers
 * (Lehner & Wettig; not part of the paper, whose plan for faster local solves
 * is multigrid).  Layer l maps chans[l] colour-vector channels to chans[l+1]:
 *   out_a(x,s) = sum_pi sum_b W_l[pi][a][b] (T_pi phi_b)(x,s)
 * over 11 paths pi: 0 identity; 1+mu: U_mu(x) phi(x+mu); 5+mu: U_mu(x-mu)^+
 * phi(x-mu) (mu = x,y,z,t); 9: phi(x,s+1); 10: phi(x,s-1) (zero outside
 * 0 <= s < Ls).  Links are the context's (Dirichlet faces included).  The first
 * and last layers have 4 channels, the spin components of a fermion; as a
 * preconditioner of the odd Schur system the network acts on the odd field
 * embedded in the full lattice (zero on even sites) and its output is
 * restricted to odd sites.  Weights are stored in BF16 with FP32 masters;
 * arithmetic is FP32.  Channel counts must be 4, 8 or 12. */
typedef struct dwf_net_s *dwf_net;

typedef struct {
    double lr, beta1, beta2, eps;  /* Adam step size and moments */
} dwf_adam;

dwf_status dwf_net_create(dwf_ctx ctx, int nlayer, const int *chans, dwf_net *out);
dwf_status dwf_net_destroy(dwf_net net);
/* number of complex weights: sum_l 11 chans[l+1] chans[l] (-1 for a null net) */
int dwf_net_num_weights(dwf_net net);
/* weights in host memory: FP32 (re, im) pairs, layer blocks back to back,
 * each block [pi][a][b] (a output, b input channel); setting resets Adam */
dwf_status dwf_net_set_weights(dwf_net net, const float *w);
dwf_status dwf_net_get_weights(dwf_net net, float *w);
/* Forward used when the network is applied as a preconditioner
 * (dwf_precond_apply, dwf_fgcr):
 *   DWF_NET_FWD_FP32       vector units, FP32 arithmetic (the default; training
 *                          always uses it)
 *   DWF_NET_FWD_MFMA_BF16  channel mixing on the matrix cores, the transported
 *                          inputs rounded to BF16 (the weights are BF16 already),
 *                          FP32 accumulation, activations between layers stored
 *                          in BF16; relative deviation from the FP32 forward at
 *                          most (1 + 2^-8)^L - 1 for L layers without
 *                          cancellation (1.6e-2 for four) */
enum { DWF_NET_FWD_FP32 = 0, DWF_NET_FWD_MFMA_BF16 = 1 };
dwf_status dwf_net_set_forward(dwf_net net, int mode);
/* out = restrict_odd(N(embed_odd(in))); canonical FP64 odd half fields */
dwf_status dwf_precond_apply(dwf_ctx ctx, dwf_net net, const double *in_odd, double *out_odd);
/* The same on internal odd half fields (layout of dwf_import) in storage
 * precisions in_prec and out_prec (DWF_F64/F32/F16/BF16; in and out distinct
 * device buffers), as FGCR applies it.  With the matrix-core forward, an FP32
 * input (or a BF16 one, for networks of two layers or more) and an FP32 or
 * BF16 output, the first layer reads the input spinor and the last writes the
 * output spinor directly (no layout passes); the result is the same as
 * through the feature layout. */
dwf_status dwf_precond_apply_internal(dwf_ctx ctx, dwf_net net, int in_prec, const void *in, int out_prec,
                                      void *out);
/* Gradients of a real loss L through y = precond(in), given grad_out =
 * dL/dRe(y) + i dL/dIm(y): grad_in the same for the input (may be NULL) and
 * grad_w (host, FP32 pairs in the weight layout, may be NULL). */
dwf_status dwf_net_backward(dwf_net net, const double *in_odd, const double *grad_out_odd, double *grad_in_odd,
                            float *grad_w);
/* One training step on nbatch pairs (b_j, x_j), canonical FP64 odd fields on
 * the device: loss = (1/nbatch) sum_j |N(b_j) - x_j|^2 / |x_j|^2, gradients by
 * the network's own backward kernels, then one Adam update of the FP32 masters
 * (skipped when opt is NULL, which evaluates the loss only). */
dwf_status dwf_net_train_step(dwf_net net, int nbatch, const double *const *b_odd, const double *const *x_odd,
                              const dwf_adam *opt, double *loss);

/* Flexible GCR(m) on the odd Schur system Mpc x_o = b~_o (o->normal = 0) or on
 * Mpc^+ Mpc x_o = Mpc^+ b~_o (o->normal = 1), right-preconditioned by net
 * (NULL: plain GCR; normal equations use N N^+).  o->mode DWF_SOLVE_F64 keeps
 * every vector in FP64; DWF_SOLVE_MIXED_F32 runs the cycle (operator, network
 * input and output, Krylov vectors) in FP32 storage with FP64 sums and folds
 * each cycle's solution into the FP64 solution, whose residual is recomputed
 * in FP64 at every restart; DWF_SOLVE_MIXED_BF16 does the same with the
 * Krylov basis (network outputs and their operator images) stored in BF16
 * and the operator applied in BF16 storage, the cycle's residual and solution
 * staying FP32 (other modes: DWF_ENOTSUP); in that mode only the images are
 * orthogonalised, and the cycle's solution update is combined at the restart
 * from the directions as the network made them, and the matrix-core network
 * reads a BF16 copy of the residual.  Restart every o->restart steps (default
 * 16, at most 64) with the residual recomputed.  Stagnation means no 10%
 * reduction of the true residual norm (the FP64 one recomputed at the
 * restarts) over max(8 m, 256) steps.  On stagnation or a non-finite residual
 * it falls back to dwf_cg in FP64 when o->fallback (the statistics then say
 * fell_back = 1).  Same source preparation and reconstruction as dwf_cg;
 * canonical FP64 full fields.  Its vectors are context workspace fields; its
 * Gram-Schmidt coefficient tables and partial sums (O(m^2) doubles plus one
 * per workgroup) are allocated and freed by each call, also while a caller
 * workspace is set, so FGCR has no entry in the workspace operations. */
dwf_status dwf_fgcr(dwf_ctx ctx, dwf_net net, const double *b_full, double *x_full, const dwf_solver_opts *o,
                    dwf_solver_stats *st);

/* ------------------------------------------------------ tile schedules */

/* Schedule selector (not a timing class): the fused stencil stages launched
 * over a batch of fields, as the multi-shift solver launches them. */
enum { DWF_SCHED_STENCIL_BATCHED = 8 };

/* Launch shape of a kernel family (DWF_K_STENCIL covers the hop and every
 * fused stencil stage on one field, DWF_SCHED_STENCIL_BATCHED the same stages
 * over a batch of fields, DWF_K_SLOCAL the fifth-dimension kernels):
 * sites_per_group 4D sites per workgroup (workgroup = Ls x sites_per_group
 * lanes, at most 256; 0 = default) and xcd_run, the number of consecutive
 * tiles each of the 8 XCDs processes before the next XCD takes over (1 = the
 * hardware's round-robin).  Results do not depend on the schedule except for
 * the order of the FP64 partial sums of fused reductions. */
dwf_status dwf_set_tile_schedule(dwf_ctx ctx, int kclass, int sites_per_group, int xcd_run);
dwf_status dwf_get_tile_schedule(dwf_ctx ctx, int kclass, int *sites_per_group, int *xcd_run);

/* Internal site order.  Internal fields store the 4D sites of a parity in
 * columns of cx x cy x cz sites (x, y, z extents; cx even) that run along t,
 * so that a sweep over one column keeps its +-t neighbours in the XCD's L2.
 * dwf_create picks a column for the lattice size (the whole 3D slice for small
 * lattices); dwf_set_site_order(ctx, 0, 0, 0) restores that choice.  Changing
 * the order invalidates every field held in the internal layout (re-import
 * them); canonical-layout calls are unaffected.  The order is the same for
 * both parities, so a half field's internal layout does not depend on its
 * parity. */
dwf_status dwf_set_site_order(dwf_ctx ctx, int cx, int cy, int cz);
dwf_status dwf_get_site_order(dwf_ctx ctx, int *cx, int *cy, int *cz);

/* Autotuner: times candidate schedules of the fused stencil in storage
 * precision prec on this context's lattice (scratch fields allocated and freed
 * by the call): every candidate once, then the four fastest and the current
 * schedule best-of-three with longer runs.  It applies the fastest, but keeps
 * the current schedule unless the winner beats it by more than 2% (timing
 * noise), and, when cache_path is not NULL, stores
 * it in a JSON cache keyed by lattice, Ls, precision and device; a later call
 * with the same key reads the cache instead of timing.  Synchronises the
 * stream.  best_ms (may be NULL) returns the time of the chosen schedule. */
dwf_status dwf_tune(dwf_ctx ctx, int prec, const char *cache_path, double *best_ms);

/* The autotuner for one operation: op DWF_TUNE_NORMAL times the normal
 * operator on one field (dwf_tune's search; nrhs must be 1) and sets the
 * DWF_K_STENCIL schedule; DWF_TUNE_BATCHED times the normal operator over a
 * batch of nrhs fields (1 <= nrhs <= 64), the multi-shift solver's launch, and
 * sets the DWF_SCHED_STENCIL_BATCHED schedule.  Cache keys carry the op and
 * nrhs (the single-field key is dwf_tune's).  Otherwise as dwf_tune. */
enum { DWF_TUNE_NORMAL = 0, DWF_TUNE_BATCHED = 1 };
dwf_status dwf_tune_op(dwf_ctx ctx, int op, int prec, int nrhs, const char *cache_path, double *best_ms);

/* ------------------------------------------------------ measurement */

/* Plain streaming copy of `bytes` bytes (a multiple of 16; 16-byte aligned
 * device pointers, non-overlapping) on the context's stream.  It reads and
 * writes each byte once and serves as the achievable-bandwidth reference of
 * the roofline and as the calibration kernel for memory counters. */
dwf_status dwf_stream_copy(dwf_ctx ctx, const void *src, void *dst, size_t bytes);

/* Bandwidth probes, the achievable-bandwidth references of the rooflines (not
 * part of the method).  kind 0: dst = a (bytes read, bytes written); 1: a is
 * read (bytes) and each workgroup writes the XOR of its part to one 16-byte
 * word of dst, which must hold 16 * min(65536, ceil(bytes / (4096 unroll)))
 * bytes; 2: dst = a XOR b (2 bytes read per byte written, the read:write mix of
 * the hop).  Each lane keeps `unroll` (1, 2, 4 or 8) independent 16-byte loads
 * in flight; nontemporal != 0 uses non-temporal loads and stores.  Device
 * pointers, 16-byte aligned; bytes a multiple of 16.  Timed as DWF_K_BLAS with
 * the bytes moved (read + written). */
dwf_status dwf_stream_probe(dwf_ctx ctx, int kind, int unroll, int nontemporal, const void *a, const void *b,
                            void *dst, size_t bytes);

/* ------------------------------------------------------ kernel statistics */

enum {
    DWF_K_DHOP = 0,     /* standalone hop kernels                           */
    DWF_K_STENCIL = 1,  /* fused Schur-complement stencil stages            */
    DWF_K_SLOCAL = 2,   /* s-local (fifth-dimension) kernels                */
    DWF_K_BLAS = 3,     /* vector updates, conversions and reductions       */
    DWF_K_NET = 4,      /* network kernels                                  */
    DWF_K_NCLASS = 5
};

/* Enable (1) or disable (0) HIP-event timing of every launch on the context's
 * stream; statistics accumulate until reset.  Each timed launch is bracketed
 * by two events, which costs a few microseconds of idle time; the mask form
 * times only the classes whose bit (1 << class) is set. */
dwf_status dwf_kernel_timing(dwf_ctx ctx, int enable);
dwf_status dwf_kernel_timing_mask(dwf_ctx ctx, int mask);
dwf_status dwf_kernel_timing_reset(dwf_ctx ctx);
/* Per kernel class: launches, summed device time (ms), summed algorithmic
 * bytes and flops, over launches whose fields have storage precision prec
 * (DWF_F64 .. DWF_BF16), or over all launches of the class (prec = -1).
 * Synchronises the stream. */
dwf_status dwf_kernel_stats(dwf_ctx ctx, int kclass, int prec, long *launches, double *ms, double *bytes,
                            double *flops);

#ifdef __cplusplus
}
#endif
#endif /* DWF_H */
