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
    double delta;      /* reliable-update threshold (<= 0: 0.1)                   */
    int x0_is_guess;   /* 1: x holds an initial guess on entry                    */
    int restart;       /* FGCR restart length m (<= 0: 16)                         */
    int normal;        /* FGCR: 1 solves the normal equations Mpc^+ Mpc, 0 Mpc    */
    int fallback;      /* FGCR: 1 falls back to CG on stagnation / NaN            */
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
 * be NULL).  mode DWF_SOLVE_F64 or DWF_SOLVE_MIXED_F32 (FP32 Krylov space with
 * FP64 refinement of every shift). */
dwf_status dwf_multishift_cg(dwf_ctx ctx, int nrhs, const double *const *b_odd, int nshift,
                             const double *shifts, double *const *x_odd, const dwf_solver_opts *o,
                             dwf_solver_stats *st);

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
 * stream; statistics accumulate until reset. */
dwf_status dwf_kernel_timing(dwf_ctx ctx, int enable);
dwf_status dwf_kernel_timing_reset(dwf_ctx ctx);
/* Per kernel class: launches, summed device time (ms), summed algorithmic
 * bytes and flops.  Synchronises the stream. */
dwf_status dwf_kernel_stats(dwf_ctx ctx, int kclass, long *launches, double *ms, double *bytes,
                            double *flops);

#ifdef __cplusplus
}
#endif
#endif /* DWF_H */
