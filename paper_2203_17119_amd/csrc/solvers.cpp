// Krylov solvers on the odd-site Schur complement.
//
//   cg_core      CG on (Mpc^+ Mpc + sigma) x = rhs in FP64, or in a low storage
//                precision with FP64 reliable updates (Sleijpen & van der Vorst;
//                mixed precision as in Clark et al.)
//   dwf_cg       red-black solve of D5 x = b: Schur source, CGNE, reconstruction
//   dwf_multishift_cg   shifted systems from one Krylov space (Jegerlehner)
//
// Scalars that the loop needs are produced on the device (fixed-order FP64
// reductions) and consumed there; the host reads back |r|^2 of every
// iteration, one iteration late, for the stopping and reliable-update
// decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "dwf_internal.h"

using namespace dwf;

namespace dwf {

// device scalar slots
enum { S_RHO = 0, S_RHONEW = 1, S_PAP = 2, S_ALPHA = 3, S_BETA = 4, S_ONE = 5, S_TMP = 6, S_ALPHA1 = 7, S_DOT = 8 };
// two more alpha slots of the CG direction ring, clear of the other solvers' slots
enum { S_ALPHA2 = 250, S_ALPHA3 = 251 };
// Re and Im of the DD-RHMC action's inner product
enum { S_DD_DOT = 246 };
static constexpr int CG_RING = 4;  // directions per pass of the solution update
static constexpr int kAlphaSlot[CG_RING] = {S_ALPHA, S_ALPHA1, S_ALPHA2, S_ALPHA3};

static double now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static int prec_of_mode(int mode)
{
    switch (mode) {
    case DWF_SOLVE_F64: return P_F64;
    case DWF_SOLVE_MIXED_F32: return P_F32;
    case DWF_SOLVE_MIXED_F16: return P_F16;
    case DWF_SOLVE_MIXED_BF16: return P_BF16;
    default: fail(DWF_EINVAL, "unknown solver mode");
    }
}

static void set_scalar(Context &c, int slot, double v)
{
    c.hscal[slot] = v;
    launch_set_scalar(c, slot, v);
}

static double norm2(Context &c, int prec, Field a, int slot = S_TMP)
{
    const int np = launch_norm2(c, prec, a);
    launch_finish(c, np, 1, slot);
    read_scalars(c, slot, 1);
    return c.hscal[slot];
}

// ap = (Mpc^+ Mpc + sigma) p ; dscal[S_PAP] = <p, ap>.  pa = A p when given.
static void normal_op(Context &c, int prec, double sigma, Field p, Field ap, Field m, bool have_pa, Field pa)
{
    if (sigma == 0.0) {
        const int np = apply_mpc(c, prec, false, p, m, true, have_pa, pa);
        launch_finish(c, np, 1, S_PAP);  // <p, Mpc^+ Mpc p> = |Mpc p|^2
        apply_mpc(c, prec, true, m, ap, false);
    } else {
        apply_mpc(c, prec, false, p, m, false, have_pa, pa);
        apply_mpc(c, prec, true, m, ap, false);
        launch_axpby(c, prec, 1.0, ap, sigma, p, ap);
        const int np = launch_dot(c, prec, p, ap);
        launch_finish(c, np, 2, S_DOT);
        launch_scalar_div(c, S_PAP, S_DOT, S_ONE);
    }
}

struct CoreStats {
    int iters = 0, reliable = 0, converged = 0;
    double rel_res = 0;
};

// Solve (Mpc^+ Mpc + sigma) x = rhs.  rhs and x are FP64 fields; x holds the
// initial guess when guess is set.  Stops when |r| <= tol |rhs| in FP64.
static CoreStats cg_core(Context &c, int mode, double sigma, Field rhs, Field x, double tol, int maxit,
                         double delta, bool guess)
{
    CoreStats st;
    const int lp = prec_of_mode(mode);
    const bool mixed = lp != P_F64;
    set_scalar(c, S_ONE, 1.0);
    const double rhs2 = norm2(c, P_F64, rhs);
    if (rhs2 == 0.0) {
        launch_zero(c, P_F64, x);
        st.converged = 1;
        return st;
    }
    const double target = tol * std::sqrt(rhs2);
    Field m64 = ws_field(c, "cg_m64", P_F64), ap64 = ws_field(c, "cg_ap64", P_F64);
    Field rh = ws_field(c, "cg_rh", P_F64);

    // r_h = rhs - A x
    auto true_residual = [&]() {
        if (!guess && st.iters == 0 && st.reliable == 0) {
            launch_copy(c, P_F64, rhs, rh);
            const int np = launch_norm2(c, P_F64, rh);
            launch_finish(c, np, 1, S_RHONEW);
        } else {
            apply_mpc(c, P_F64, false, x, m64, false);
            apply_mpc(c, P_F64, true, m64, ap64, false);
            if (sigma != 0.0) launch_axpby(c, P_F64, 1.0, ap64, sigma, x, ap64);
            const int np = launch_residual(c, rhs, ap64, rh);
            launch_finish(c, np, 1, S_RHONEW);
        }
        read_scalars(c, S_RHONEW, 1);
        return c.hscal[S_RHONEW];
    };
    if (!guess) launch_zero(c, P_F64, x);

    const int xp = accum_prec(lp);
    Field r = mixed ? ws_field(c, "cg_rl", lp) : rh;
    Field xl = mixed ? ws_field(c, "cg_xl", xp) : x;
    // a ring of direction buffers: the current p, and up to three older ones
    // whose solution updates are still pending
    Field pbuf[CG_RING];
    for (int q = 0; q < CG_RING; q++) pbuf[q] = ws_field(c, "cg_p" + std::to_string(q), lp);
    Field pa = ws_field(c, "cg_pa", lp);
    int cur = 0;
    Field m = mixed ? ws_field(c, "cg_m", lp) : m64, ap = mixed ? ws_field(c, "cg_ap", lp) : ap64;

    double rho = true_residual();
    if (mixed) {
        launch_convert(c, P_F64, rh, lp, r);
        launch_zero(c, xp, xl);
    }
    // p = r, pa = A p  (via p = r + 0 p)
    set_scalar(c, S_BETA, 0.0);
    launch_zero(c, lp, pbuf[0]);
    launch_cg_update_p(c, lp, r, pbuf[0], pbuf[0], pa, S_BETA);
    set_scalar(c, S_RHO, rho);
    double rmax = std::sqrt(rho);
    if (std::sqrt(rho) <= target) {
        st.converged = 1;
        st.rel_res = std::sqrt(rho / rhs2);
        return st;
    }
    const int maxi = maxit > 0 ? maxit : 100000;
    // Unshifted systems fuse the residual update into the last stencil stage
    // (r -= alpha Mpc^+ Mpc p without storing the product) and defer the
    // solution update x += alpha p to a p-update kernel, which reads p anyway.
    // Every fourth p-update folds four iterations' updates into one pass over
    // x: the older directions stay in the ring until then, each with its alpha
    // in the slot of its ring position.  Before a reliable update or the exit
    // the pending updates are applied on their own.
    const bool fused = sigma == 0.0;
    int npend = 0;  // older iterations whose solution updates are pending
    auto ring = [&](int back) { return (cur - back + CG_RING) % CG_RING; };
    // The host learns each iteration's residual norm one iteration late. The
    // reduction of iteration k writes the norm to a ring slot in host memory
    // as well, and the host waits for it only after it has queued iteration
    // k + 1, so the device never idles on the round trip. A reliable update or
    // an exit that the norm of iteration k calls for follows iteration k + 1;
    // it then reads that iteration's own norm.
    int unread = -1;  // iteration whose norm the host has not read yet
    // A low-precision recurrence drifts from the true residual with every
    // iteration; on an ill-conditioned operator the residual may fall by the
    // factor delta only after hundreds of them.  A reliable update is also due
    // after kMaxSinceUpdate iterations without one.
    static constexpr int kMaxSinceUpdate = 150;
    int since_update = 0;
    auto norm_of = [&](int k) {
        HIPCHECK(hipEventSynchronize(c.cg_ev[k & 1]));
        const double v = *(volatile double *)(c.hring + (k & 1));
        if (!std::isfinite(v)) fail(DWF_ENOCONV, "CG breakdown: non-finite residual");
        return v;
    };
    while (true) {
        const Field p = pbuf[cur];
        const int aslot = kAlphaSlot[cur];
        if (fused) {
            const int npm = apply_mpc(c, lp, false, p, m, true, true, pa);
            // <p, Mpc^+ Mpc p> = |Mpc p|^2, and alpha = rho / <p, Mpc^+ Mpc p>
            launch_finish(c, npm, 1, S_PAP, nullptr, aslot, S_RHO);
            const int np = apply_mpc(c, lp, true, m, r, false, false, Field{}, 1, 0, aslot);
            launch_finish(c, np, 1, S_RHONEW, c.dring + (st.iters & 1));
        } else {
            normal_op(c, lp, sigma, p, ap, m, true, pa);
            launch_scalar_div(c, aslot, S_RHO, S_PAP);
            const int np = launch_cg_update_xr(c, lp, xl, r, p, ap, aslot);
            launch_finish(c, np, 1, S_RHONEW, c.dring + (st.iters & 1));
        }
        const int k = st.iters++;
        HIPCHECK(hipEventRecord(c.cg_ev[k & 1], c.stream));
        // the check that the previous iteration's norm asks for
        since_update++;
        bool check = st.iters >= maxi || (mixed && since_update >= kMaxSinceUpdate);
        if (unread >= 0) {
            const double rn = std::sqrt(norm_of(unread));
            check = check || rn <= target || (mixed && rn < delta * rmax);
        }
        unread = k;
        bool x_pending = fused;  // x += alpha p of this iteration not yet applied
        auto flush = [&]() {
            for (int back = npend; back >= 1; back--)
                launch_axpy_dev(c, lp, xl, pbuf[ring(back)], kAlphaSlot[ring(back)]);
            if (x_pending) launch_axpy_dev(c, lp, xl, p, aslot);
            npend = 0;
            x_pending = false;
        };
        bool done = false;
        if (check) {
            double rho1 = norm_of(k);
            unread = -1;
            if (mixed) {
                // reliable update: fold the low-precision solution into x and
                // recompute the residual exactly
                flush();
                launch_accumulate_low(c, xp, x, xl);
                rho1 = true_residual();
                launch_convert(c, P_F64, rh, lp, r);
                rmax = std::sqrt(rho1);
                st.reliable++;
                since_update = 0;
            }
            done = std::sqrt(rho1) <= target;
        }
        if (done || st.iters >= maxi) {
            flush();
            if (done) st.converged = 1;
            break;
        }
        launch_cg_beta(c, S_BETA, S_RHO, S_RHONEW);
        // The new direction goes to the next ring position. It holds no pending
        // direction, or the oldest one, whose update this kernel applies first.
        const int nxt = (cur + 1) % CG_RING;
        if (x_pending && npend == CG_RING - 1) {
            CgOlder older;
            for (int back = npend; back >= 1; back--) {
                older.dir[older.n] = pbuf[ring(back)];
                older.slot[older.n++] = kAlphaSlot[ring(back)];
            }
            launch_cg_update_p(c, lp, r, p, pbuf[nxt], pa, S_BETA, xl, aslot, older);
            npend = 0;
        } else {
            launch_cg_update_p(c, lp, r, p, pbuf[nxt], pa, S_BETA);
            npend = x_pending ? npend + 1 : 0;
        }
        cur = nxt;
    }
    if (mixed && !st.converged) launch_accumulate_low(c, xp, x, xl);
    // final FP64 check
    guess = true;
    const double rf = true_residual();
    st.rel_res = std::sqrt(rf / rhs2);
    st.converged = st.rel_res <= tol * 1.0000001 ? 1 : 0;
    return st;
}

static void fill_opts(const dwf_solver_opts *o, double &tol, int &maxit, int &mode, double &delta, bool &guess)
{
    tol = (o && o->tol > 0) ? o->tol : 1e-8;
    maxit = (o && o->maxit > 0) ? o->maxit : 100000;
    mode = o ? o->mode : DWF_SOLVE_F64;
    delta = (o && o->delta > 0) ? o->delta : 0.1;
    guess = o && o->x0_is_guess;
    prec_of_mode(mode);
}

}  // namespace dwf

extern "C" {

dwf_status dwf_cg(dwf_ctx ctx, const double *b_full, double *x_full, const dwf_solver_opts *o, dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!b_full || !x_full) fail(DWF_EINVAL, "null field pointer");
    dwf::Context &c = *ctx;
    double tol, delta;
    int maxit, mode;
    bool guess;
    fill_opts(o, tol, maxit, mode, delta, guess);
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t0 = now();
    Field be = ws_field(c, "sv_be", P_F64), bo = ws_field(c, "sv_bo", P_F64);
    Field bt = ws_field(c, "sv_bt", P_F64), rhs = ws_field(c, "sv_rhs", P_F64);
    Field xo = ws_field(c, "sv_xo", P_F64), xe = ws_field(c, "sv_xe", P_F64);
    Field t1 = ws_field(c, "sv_t1", P_F64), t2 = ws_field(c, "sv_t2", P_F64);
    launch_import(c, P_F64, b_full, be, 1, 0);
    launch_import(c, P_F64, b_full, bo, 1, 1);
    if (guess) launch_import(c, P_F64, x_full, xo, 1, 1);
    // b~_o = b_o - Moe Mee^-1 b_e = b_o + (1/2) H_oe A Mee^-1 b_e
    launch_slocal(c, P_F64, SL_E1, be, t1);
    StencilSpec sp;
    sp.out_parity = 1;
    sp.self = true;
    sp.s0 = 1.0;
    sp.s1 = 0.0;
    sp.tau = 0.5;
    launch_stencil(c, P_F64, sp, t1, bo, bt);
    // normal-equation right-hand side Mpc^+ b~
    apply_mpc(c, P_F64, true, bt, rhs, false);
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t1w = now();
    CoreStats cs = cg_core(c, mode, 0.0, rhs, xo, tol, maxit, delta, guess);
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t2w = now();
    // x_e = Mee^-1 (b_e - Meo x_o) = Mee^-1 (b_e + (1/2) H_eo A x_o)
    launch_slocal(c, P_F64, SL_A, xo, t1);
    sp = StencilSpec{};
    sp.out_parity = 0;
    sp.self = true;
    sp.s0 = 1.0;
    sp.tau = 0.5;
    launch_stencil(c, P_F64, sp, t1, be, t2);
    launch_slocal(c, P_F64, SL_MINV, t2, xe);
    launch_export(c, P_F64, xe, x_full, 1, 0);
    launch_export(c, P_F64, xo, x_full, 1, 1);
    // residuals in FP64
    apply_mpc(c, P_F64, false, xo, t1, false);
    launch_axpby(c, P_F64, 1.0, bt, -1.0, t1, t1);  // b~ - Mpc x
    const double bt2 = dwf::norm2(c, P_F64, bt, S_TMP);
    const double rs2 = dwf::norm2(c, P_F64, t1, S_TMP);
    apply_mpc(c, P_F64, true, t1, t2, false);
    const double rn2 = dwf::norm2(c, P_F64, t2, S_TMP);
    const double rhs2 = dwf::norm2(c, P_F64, rhs, S_TMP);
    // D5 x on both parities: Mooee x_p - (1/2) H_{p,1-p} A x_{1-p}
    Field ax = ws_field(c, "sv_ax", P_F64);
    double r2 = 0, b2 = 0;
    for (int par = 0; par < 2; par++) {
        Field xp = par ? xo : xe, xq = par ? xe : xo, bp = par ? bo : be;
        launch_slocal(c, P_F64, SL_A, xq, ax);
        StencilSpec d5;
        d5.out_parity = par;
        d5.self = true;
        d5.s0 = c.d;
        d5.s1 = c.e;
        d5.tau = -0.5;
        launch_stencil(c, P_F64, d5, ax, xp, t2);
        launch_axpby(c, P_F64, 1.0, bp, -1.0, t2, t2);
        r2 += dwf::norm2(c, P_F64, t2, S_TMP);
        b2 += dwf::norm2(c, P_F64, bp, S_TMP);
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t3w = now();
    if (st) {
        st->iters = cs.iters;
        st->reliable_updates = cs.reliable;
        st->converged = cs.converged;
        st->fell_back = 0;
        st->res_normal = rhs2 > 0 ? std::sqrt(rn2 / rhs2) : 0.0;
        st->res_schur = bt2 > 0 ? std::sqrt(rs2 / bt2) : 0.0;
        st->res_full = b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
        st->seconds = t3w - t0;
        st->t_prep = t1w - t0;
        st->t_solve = t2w - t1w;
        st->t_final = t3w - t2w;
    }
    return cs.converged ? DWF_OK : DWF_ENOCONV;
    DWF_API_END
}

}  // extern "C"

// ---------------------------------------------------------- multi-shift CG

namespace dwf {

// device state of the batched multi-shift solver: per-rhs scalars, per
// (shift, rhs) recurrences and two coefficient sets, the shifts, flags.  The
// buffer is sized for the largest batch (64 x 64), so that one workspace
// buffer serves every call.
static size_t ms_state_bytes(int nrhs, int nshift)
{
    (void)nrhs;
    (void)nshift;
    const size_t nq = 64 * 64;
    return sizeof(double) * (7 * 64 + 2 * nq + 4 * nq + 64 + 4 * nq) + sizeof(int) * 2 * nq;
}

// Workspace buffers of cg_core in a mode (keys as its ws_field calls)
static void plan_cg_core(std::vector<WsKey> &k, int mode)
{
    const int lp = prec_of_mode(mode), xp = accum_prec(lp);
    const bool mixed = lp != P_F64;
    for (const char *n : {"cg_m64", "cg_ap64", "cg_rh", "mpc_y", "mpc_ta"}) k.push_back({n, P_F64, 0, 0});
    for (int q = 0; q < CG_RING; q++) k.push_back({"cg_p" + std::to_string(q), lp, 0, 0});
    k.push_back({"cg_pa", lp, 0, 0});
    if (mixed) {
        k.push_back({"cg_rl", lp, 0, 0});
        k.push_back({"cg_xl", xp, 0, 0});
        k.push_back({"cg_m", lp, 0, 0});
        k.push_back({"cg_ap", lp, 0, 0});
        k.push_back({"mpc_y", lp, 0, 0});
    }
}

std::vector<WsKey> plan_cg(int mode)
{
    std::vector<WsKey> k;
    for (const char *n : {"sv_be", "sv_bo", "sv_bt", "sv_rhs", "sv_xo", "sv_xe", "sv_t1", "sv_t2", "sv_ax"})
        k.push_back({n, P_F64, 0, 0});
    plan_cg_core(k, mode);
    return k;
}

std::vector<WsKey> plan_multishift(int mode, int nrhs, int nshift)
{
    const int lp = prec_of_mode(mode);
    const int nq = nrhs * nshift;
    std::vector<WsKey> k;
    for (const char *n : {"ms_B", "ms_R", "ms_AP", "ms_M"}) k.push_back({n, lp, nrhs, 0});
    for (const char *n : {"ms_X", "ms_P", "ms_P2"}) k.push_back({n, lp, nq, 0});
    // the batched operator's intermediates (one field when nrhs == 1)
    k.push_back({"mpc_y", lp, nrhs, 0});
    k.push_back({"mpc_ta", lp, nrhs, 0});
    for (const char *n : {"ms_b64", "ms_x64", "ms_t1", "ms_t2"}) k.push_back({n, P_F64, 0, 0});
    k.push_back({"ms_state", -1, 0, ms_state_bytes(nrhs, nshift)});
    // the FP64 residual check and the refinement of systems that missed the
    // tolerance: batched corrections, then the single-system CG
    if (lp != P_F64)
        for (const char *n : {"msr_E", "msr_D"}) k.push_back({n, lp, nrhs, 0});
    plan_cg_core(k, mode);
    return k;
}

}  // namespace dwf

namespace dwf {

// Receives the FP64 solution of system (rhs j, shift k) in the internal layout
// once it has met its tolerance (or the iteration limit); the field is reused
// for the next system, so the sink consumes it on the stream before returning.
using MsSink = std::function<void(int j, int k, Field x64)>;

// Buffers of one multi-shift CG run: per right-hand side (capacity >= nrhs) the
// sources B, residuals R, A p, the operator's intermediates M, Y, TA; per
// member (shift k, rhs j: member k nrhs + j, capacity >= nrhs nshift) the
// solutions X and two direction sets (the current directions, and the new
// ones, which hold the previous directions while their solution updates are
// pending).  All use the batch stride of their precision.
struct MsBufs {
    Field B, R, AP, M, Y, TA;
    Field X, P[2];
};

// Multi-shift CG iterations on (Mpc^+ Mpc + shifts[k]) X_{k,j} = B_j in storage
// precision lp, from X = 0, until |r_{j,k}| <= rtol[j] |B_j| for every member or
// maxi iterations.  its[q]: iterations of member q; act[q]: still active at
// the end.  The host reads the members' activity every poll iterations.
// Returns the iterations run.
static int ms_krylov(Context &c, int lp, int nrhs, int nshift, const double *shifts, const MsBufs &bf,
                     const double *rtol, int maxi, int poll, std::vector<int> &its, std::vector<int> &act)
{
    const long stride = batch_stride(c, lp);
    const int nq = nrhs * nshift;
    int kmin = 0;
    for (int k = 1; k < nshift; k++)
        if (shifts[k] < shifts[kmin]) kmin = k;
    // device state
    double *db = (double *)ws_raw(c, "ms_state", ms_state_bytes(nrhs, nshift));
    MsState s;
    s.rho = db;
    s.pap = db + nrhs;
    s.alpha = db + 2 * nrhs;
    s.alpha_old = db + 3 * nrhs;
    s.beta_old = db + 4 * nrhs;
    s.target = db + 5 * nrhs;
    double *rho_new = db + 6 * nrhs;
    s.zeta = db + 7 * nrhs;
    s.zeta_old = s.zeta + nq;
    s.coef = s.zeta_old + nq;
    s.shifts = s.coef + 4 * nq;
    double *coefs[2] = {s.coef, s.shifts + nshift};  // this and the previous iteration's coefficients
    s.active = (int *)(coefs[1] + 4 * nq);
    s.iters = s.active + nq;
    {
        std::vector<double> h(7 * nrhs + 6 * nq + nshift + 4 * nq, 0.0);
        std::vector<int> hi(2 * nq, 0);
        ms_launch_norm2(c, lp, bf.B, nrhs, stride, c.dscal + 16);
        read_scalars(c, 16, nrhs);
        for (int j = 0; j < nrhs; j++) {
            h[j] = c.hscal[16 + j];                              // rho
            h[3 * nrhs + j] = 1.0;                               // alpha_old
            h[5 * nrhs + j] = rtol[j] * std::sqrt(c.hscal[16 + j]);  // target
        }
        for (int q = 0; q < nq; q++) h[7 * nrhs + q] = h[7 * nrhs + nq + q] = 1.0;  // zeta, zeta_old
        for (int k = 0; k < nshift; k++) h[7 * nrhs + 6 * nq + k] = shifts[k];
        for (int q = 0; q < nq; q++) hi[q] = 1;
        HIPCHECK(hipMemcpy(db, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s.active, hi.data(), hi.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    for (int j = 0; j < nrhs; j++) launch_copy(c, lp, member(bf.B, j, stride), member(bf.R, j, stride));
    for (int q = 0; q < nq; q++) {
        launch_zero(c, lp, member(bf.X, q, stride));
        launch_copy(c, lp, member(bf.B, q % nrhs, stride), member(bf.P[0], q, stride));
    }
    // the operator's first factor (b + c P5) of the carrier's directions; the
    // step kernel keeps it up to date for the new directions
    launch_slocal(c, lp, SL_A, bf.B, bf.TA, nrhs, stride);
    act.assign(nq, 1);
    its.assign(nq, 0);
    int it = 0, cur = 0;  // bf.P[cur] holds the current directions
    while (it < maxi) {
        // AP = Mpc^+ Mpc p of the carrier; its shift enters the dot product
        // and the residual update
        const Field Pbase = member(bf.P[cur], kmin * nrhs, stride);
        apply_mpc(c, lp, false, Pbase, bf.M, false, true, bf.TA, nrhs, stride, -1, Field{}, bf.Y);
        apply_mpc(c, lp, true, bf.M, bf.AP, false, false, Field{}, nrhs, stride, -1, Field{}, bf.Y);
        ms_launch_redot(c, lp, Pbase, bf.AP, nrhs, stride, s.pap, shifts[kmin]);
        it++;
        MsState si = s;
        si.coef = coefs[cur];
        ms_launch_step(c, lp, si, bf.R, bf.AP, bf.X, bf.P[cur], bf.P[1 - cur], coefs[1 - cur], nrhs, nshift, kmin,
                       stride, rho_new, it, Pbase, shifts[kmin], bf.TA);
        cur = 1 - cur;
        if (it % poll == 0 || it == maxi) {
            HIPCHECK(hipMemcpyAsync(act.data(), s.active, nq * sizeof(int), hipMemcpyDeviceToHost, c.stream));
            HIPCHECK(hipStreamSynchronize(c.stream));
            int n = 0;
            for (int a : act) n += a;
            if (n == 0) break;
        }
    }
    // an odd last iteration left its solution updates pending
    if (it % 2 == 1) ms_launch_flush(c, lp, bf.X, bf.P[1 - cur], coefs[1 - cur], nrhs, nshift, stride);
    HIPCHECK(hipMemcpy(its.data(), s.iters, nq * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(act.data(), s.active, nq * sizeof(int), hipMemcpyDeviceToHost));
    for (int q = 0; q < nq; q++)
        if (act[q]) its[q] = it;
    return it;
}

// Multi-shift CG on (Mpc^+ Mpc + shifts[k]) x_{j,k} = b_j for canonical FP64
// odd fields b_odd[j] (device).  Arguments are validated by the caller.
// Returns true when every system met the tolerance in FP64.
//
// Every solution's residual is then recomputed in FP64.  In MIXED_F32 the
// solutions are refined by defect correction, batched over the right-hand
// sides of one shift: the FP64 residuals of the systems that missed the
// tolerance are solved together by the same CG iteration (one shift) in FP32
// storage, warm-started in the sense that only the correction is solved for,
// and the corrections accumulate in a second FP32 term beside the first
// solve's solution (x = X + E, summed in FP64), so that the solution is not
// limited by FP32 rounding of x itself.  A system still missing the tolerance
// after kRefinePasses corrections is finished by the single-system mixed CG.
static bool ms_solve(Context &c, int nrhs, const double *const *b_odd, int nshift, const double *shifts,
                     const MsSink &sink, const dwf_solver_opts *o, dwf_solver_stats *st)
{
    constexpr int kRefinePasses = 4;
    double tol, delta;
    int maxit, mode;
    bool guess;
    fill_opts(o, tol, maxit, mode, delta, guess);
    if (mode != DWF_SOLVE_F64 && mode != DWF_SOLVE_MIXED_F32)
        fail(DWF_ENOTSUP, "multi-shift mode must be F64 or MIXED_F32");
    const int lp = prec_of_mode(mode);
    const bool mixed = lp != P_F64;
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t0 = now();
    const long stride = batch_stride(c, lp);
    const int nq = nrhs * nshift;
    MsBufs bf;
    bf.B = ws_batch(c, "ms_B", lp, nrhs);
    bf.R = ws_batch(c, "ms_R", lp, nrhs);
    bf.AP = ws_batch(c, "ms_AP", lp, nrhs);
    bf.M = ws_batch(c, "ms_M", lp, nrhs);
    bf.Y = ws_batch(c, "mpc_y", lp, nrhs);
    bf.TA = ws_batch(c, "mpc_ta", lp, nrhs);
    bf.X = ws_batch(c, "ms_X", lp, nq);
    bf.P[0] = ws_batch(c, "ms_P", lp, nq);
    bf.P[1] = ws_batch(c, "ms_P2", lp, nq);
    Field b64 = ws_field(c, "ms_b64", P_F64), x64 = ws_field(c, "ms_x64", P_F64);
    std::vector<double> b2(nrhs);
    for (int j = 0; j < nrhs; j++) {
        launch_import(c, P_F64, b_odd[j], b64, 0, 0);
        b2[j] = norm2(c, P_F64, b64);
        launch_convert(c, P_F64, b64, lp, member(bf.B, j, stride));
    }
    const int maxi = maxit > 0 ? maxit : 100000;
    std::vector<int> its, act;
    const std::vector<double> rtol(nrhs, tol);
    ms_krylov(c, lp, nrhs, nshift, shifts, bf, rtol.data(), maxi, 8, its, act);
    const double t1 = now();
    // FP64 true residual of every (rhs, shift), and the refinement of the
    // systems that missed the tolerance
    Field t1f = ws_field(c, "ms_t1", P_F64), t2f = ws_field(c, "ms_t2", P_F64);
    // refinement: the first solve's sources and direction sets are free now;
    // E (corrections so far) and D (this pass's corrections) per rhs
    MsBufs rb = bf;
    Field E, D;
    if (mixed) {
        E = ws_batch(c, "msr_E", lp, nrhs);
        D = ws_batch(c, "msr_D", lp, nrhs);
        rb.X = D;
    }
    // x64 = X_q (+ E_j): the solution of system (j, k) in FP64
    auto assemble = [&](int j, int k, bool with_e) {
        launch_convert(c, lp, member(bf.X, k * nrhs + j, stride), P_F64, x64);
        if (with_e) {
            launch_convert(c, lp, member(E, j, stride), P_F64, t1f);
            launch_axpby(c, P_F64, 1.0, x64, 1.0, t1f, x64);
        }
    };
    // t2f = b_j - (Mpc^+ Mpc + shift) x64; returns |t2f| / |b_j|
    auto residual = [&](int j, double shift) {
        launch_import(c, P_F64, b_odd[j], b64, 0, 0);
        apply_mpc(c, P_F64, false, x64, t1f, false);
        apply_mpc(c, P_F64, true, t1f, t2f, false);
        launch_axpby(c, P_F64, 1.0, t2f, shift, x64, t2f);
        launch_axpby(c, P_F64, 1.0, b64, -1.0, t2f, t2f);
        return std::sqrt(norm2(c, P_F64, t2f) / b2[j]);
    };
    bool all_ok = true;
    std::vector<int> extra(nrhs);
    std::vector<double> res(nrhs);
    for (int k = 0; k < nshift; k++) {
        std::fill(extra.begin(), extra.end(), 0);
        std::vector<int> todo;
        for (int j = 0; j < nrhs; j++) todo.push_back(j);
        bool with_e = false;
        for (int pass = 0; !todo.empty(); pass++) {
            std::vector<int> fails;
            std::vector<double> rt;
            for (int j : todo) {
                assemble(j, k, with_e);
                res[j] = b2[j] > 0 ? residual(j, shifts[k]) : 0.0;
                if (res[j] > tol && mixed && pass < kRefinePasses) {
                    // the correction's source, and its relative target: 90% of the
                    // tolerance (the FP32 recurrence tracks the FP64 residual of the
                    // correction to about 1e-7 of |r|), not below what FP32
                    // storage resolves
                    launch_convert(c, P_F64, t2f, lp, member(rb.B, (int)fails.size(), stride));
                    rt.push_back(std::max(0.9 * tol / res[j], 1e-5));
                    fails.push_back(j);
                    continue;
                }
                if (res[j] > tol) {
                    // finish with the single-system CG, warm-started at x64
                    launch_import(c, P_F64, b_odd[j], b64, 0, 0);
                    CoreStats cs = cg_core(c, mode, shifts[k], b64, x64, tol, maxi, delta, true);
                    extra[j] += cs.iters;
                    res[j] = cs.rel_res;
                }
                sink(j, k, x64);
                const bool ok = res[j] <= tol * 1.0000001;
                all_ok = all_ok && ok;
                if (st) {
                    const int q = k * nrhs + j;
                    dwf_solver_stats &sv = st[j * nshift + k];
                    sv = dwf_solver_stats{};
                    sv.iters = its[q] + extra[j];
                    sv.reliable_updates = extra[j];
                    sv.converged = ok;
                    sv.res_normal = res[j];
                    sv.t_solve = t1 - t0;
                }
            }
            if (fails.empty()) break;
            const int nf = (int)fails.size();
            std::vector<int> its2, act2;
            // short solves: the activity is read every second iteration
            ms_krylov(c, lp, nf, 1, &shifts[k], rb, rt.data(), maxi, 2, its2, act2);
            for (int i = 0; i < nf; i++) {
                const int j = fails[i];
                if (!with_e) launch_zero(c, lp, member(E, j, stride));
                launch_axpby(c, lp, 1.0, member(E, j, stride), 1.0, member(D, i, stride), member(E, j, stride));
                extra[j] += its2[i];
            }
            with_e = true;
            todo = fails;
        }
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t2 = now();
    if (st)
        for (int q = 0; q < nq; q++) {
            st[q].t_final = t2 - t1;
            st[q].seconds = t2 - t0;
        }
    return all_ok;
}

static void check_shifts(int nshift, const double *shifts)
{
    for (int k = 0; k < nshift; k++)
        if (!(shifts[k] >= 0.0) || !std::isfinite(shifts[k])) fail(DWF_EINVAL, "shifts must be finite and >= 0");
}

}  // namespace dwf

extern "C" dwf_status dwf_multishift_cg(dwf_ctx ctx, int nrhs, const double *const *b_odd, int nshift,
                                        const double *shifts, double *const *x_odd, const dwf_solver_opts *o,
                                        dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (nrhs < 1 || nrhs > 64 || nshift < 1 || nshift > 64) fail(DWF_EINVAL, "need 1 <= nrhs, nshift <= 64");
    if (!b_odd || !x_odd || !shifts) fail(DWF_EINVAL, "null pointer");
    check_shifts(nshift, shifts);
    for (int j = 0; j < nrhs; j++) {
        if (!b_odd[j]) fail(DWF_EINVAL, "null right-hand side");
        for (int k = 0; k < nshift; k++)
            if (!x_odd[j * nshift + k]) fail(DWF_EINVAL, "null solution pointer");
    }
    dwf::Context &c = *ctx;
    if (o && o->tile_sb != 0) {
        const int lp = prec_of_mode(o->mode);
        if (o->tile_sb == -1) {
            HIPCHECK(hipStreamSynchronize(c.stream));
            const dwf_status ts = dwf_tune_op(ctx, DWF_TUNE_BATCHED, lp, nrhs, nullptr, nullptr);
            if (ts != DWF_OK) return ts;
        } else {
            if (o->tile_sb < 0 || (long)o->tile_sb * c.Ls > 256 || o->tile_run < 1 || o->tile_run > (1 << 20))
                fail(DWF_EINVAL, "tile_sb * Ls must be <= 256 and tile_run in [1, 2^20]");
            c.cfg_stencil_batch.sb = o->tile_sb;
            c.cfg_stencil_batch.run = o->tile_run;
        }
    }
    auto sink = [&](int j, int k, Field x64) { launch_export(c, P_F64, x64, x_odd[j * nshift + k], 0, 0); };
    if (!ms_solve(c, nrhs, b_odd, nshift, shifts, sink, o, st)) return DWF_ENOCONV;
    DWF_API_END
}

extern "C" dwf_status dwf_workspace_bytes(dwf_ctx ctx, int op, int mode, int nrhs, int nshift, size_t *bytes)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!bytes) fail(DWF_EINVAL, "null bytes");
    dwf::Context &c = *ctx;
    std::vector<WsKey> plan;
    switch (op) {
    case DWF_OP_CG: plan = plan_cg(mode); break;
    case DWF_OP_MULTISHIFT:
    case DWF_OP_RATIONAL:
        if (mode != DWF_SOLVE_F64 && mode != DWF_SOLVE_MIXED_F32)
            fail(DWF_ENOTSUP, "multi-shift mode must be F64 or MIXED_F32");
        if (op == DWF_OP_RATIONAL) nrhs = 1;
        if (nrhs < 1 || nrhs > 64 || nshift < 1 || nshift > 64) fail(DWF_EINVAL, "need 1 <= nrhs, nshift <= 64");
        plan = plan_multishift(mode, nrhs, nshift);
        if (op == DWF_OP_RATIONAL) plan.push_back({"ra_acc", P_F64, 0, 0});
        break;
    case DWF_OP_SCHUR_APPLY:
        for (const char *n : {"io_a", "io_b", "mpc_y", "mpc_ta"}) plan.push_back({n, P_F64, 0, 0});
        break;
    case DWF_OP_BOUNDARY: {
        // the solves on this context, and the boundary operators' own fields
        plan = plan_cg(mode);
        for (const char *n : {"bd_x0", "bd_x1", "bd_y0", "bd_y1", "bd_z0", "bd_z1", "bd_ax", "bd_pt"})
            plan.push_back({n, P_F64, 0, 0});
        const size_t cbytes = (size_t)2 * c.n5h * 12 * 2 * sizeof(double);
        plan.push_back({"bd_can0", -1, 0, cbytes});
        plan.push_back({"bd_can1", -1, 0, cbytes});
        break;
    }
    default: fail(DWF_EINVAL, "unknown operation");
    }
    *bytes = ws_plan_bytes(c, plan);
    DWF_API_END
}

// ------------------------------------------------------- rational functions
//
// r(A) v = a0 v + sum_k alpha_k (A + beta_k)^-1 v with A = Mpc^+ Mpc: one
// multi-shift solve with the shifts beta_k, the solutions summed on the
// device as they are produced.  The one-flavour actions of DD-RHMC apply the
// fractional powers x^{1/4} and x^{-1/2} of the normal operators this way
// (Sec. 2.3.1).

namespace dwf {

static void check_rational(const dwf_rational *r)
{
    if (!r || !r->alpha || !r->beta) fail(DWF_EINVAL, "null rational function");
    if (r->n < 1 || r->n > 64) fail(DWF_EINVAL, "rational function needs 1 <= n <= 64 poles");
    if (!std::isfinite(r->a0)) fail(DWF_EINVAL, "non-finite a0");
    for (int k = 0; k < r->n; k++)
        if (!std::isfinite(r->alpha[k])) fail(DWF_EINVAL, "non-finite alpha");
    check_shifts(r->n, r->beta);
}

// acc = r(A) in, with in a canonical FP64 odd field and acc an internal FP64
// field; st (may be NULL) gets the worst system's statistics.
static bool rational_core(Context &c, const dwf_rational *r, const double *in_odd, Field acc,
                          const dwf_solver_opts *o, dwf_solver_stats *st)
{
    launch_import(c, P_F64, in_odd, acc, 0, 0);
    launch_axpby(c, P_F64, r->a0, acc, 0.0, acc, acc);
    auto sink = [&](int, int k, Field x64) { launch_axpby(c, P_F64, 1.0, acc, r->alpha[k], x64, acc); };
    std::vector<dwf_solver_stats> per(r->n);
    const bool ok = ms_solve(c, 1, &in_odd, r->n, r->beta, sink, o, per.data());
    if (st) {
        dwf_solver_stats w = per[0];
        int conv = 1;
        for (const auto &s : per) {
            if (s.iters > w.iters) w = s;
            conv = conv && s.converged;
        }
        w.converged = conv;
        *st = w;
    }
    return ok;
}

}  // namespace dwf

extern "C" dwf_status dwf_rational_apply(dwf_ctx ctx, const dwf_rational *r, const double *in_odd, double *out_odd,
                                         const dwf_solver_opts *o, dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!in_odd || !out_odd) fail(DWF_EINVAL, "null field pointer");
    check_rational(r);
    dwf::Context &c = *ctx;
    Field acc = ws_field(c, "ra_acc", P_F64);
    const bool ok = rational_core(c, r, in_odd, acc, o, st);
    launch_export(c, P_F64, acc, out_odd, 0, 0);
    HIPCHECK(hipStreamSynchronize(c.stream));
    if (!ok) return DWF_ENOCONV;
    DWF_API_END
}

// S = phi^+ r_q(A_d) r_m(A) r_q(A_d) phi = <psi, r_m(A) psi>, psi = r_q(A_d) phi
// (r_q(A_d) is Hermitian).  psi passes from the Dirichlet context to the other
// in the canonical layout, in a workspace field of the Dirichlet context.
extern "C" dwf_status dwf_ddrhmc_action(dwf_ctx ctx, dwf_ctx ctx_dirichlet, const dwf_rational *r_quarter,
                                        const dwf_rational *r_minus_half, const double *phi_odd,
                                        const dwf_solver_opts *o, double *action, dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx || !ctx_dirichlet) fail(DWF_EINVAL, "null context");
    if (!phi_odd || !action) fail(DWF_EINVAL, "null pointer");
    check_rational(r_quarter);
    check_rational(r_minus_half);
    dwf::Context &c = *ctx, &cd = *ctx_dirichlet;
    for (int mu = 0; mu < 4; mu++)
        if (c.L[mu] != cd.L[mu]) fail(DWF_EINVAL, "contexts of different lattices");
    if (c.Ls != cd.Ls || c.p.b != cd.p.b || c.p.c != cd.p.c || c.p.M5 != cd.p.M5 || c.p.mf != cd.p.mf)
        fail(DWF_EINVAL, "contexts of different operator parameters");
    if (c.device != cd.device) fail(DWF_EINVAL, "contexts on different devices");
    // psi = r_q(A_d) phi, exported to a canonical buffer that the other context reads
    Field accd = ws_field(cd, "ra_acc", P_F64);
    Field canon = ws_field(cd, "dd_psi", P_F64);
    const bool ok1 = rational_core(cd, r_quarter, phi_odd, accd, o, st);
    launch_export(cd, P_F64, accd, (double *)canon.data, 0, 0);
    HIPCHECK(hipStreamSynchronize(cd.stream));
    // chi = r_m(A) psi ; S = Re <psi, chi>
    Field acc = ws_field(c, "ra_acc", P_F64), psi = ws_field(c, "dd_psi_in", P_F64);
    const bool ok2 = rational_core(c, r_minus_half, (const double *)canon.data, acc, o, st ? st + 1 : nullptr);
    launch_import(c, P_F64, (const double *)canon.data, psi, 0, 0);
    const int np = launch_dot(c, P_F64, psi, acc);
    launch_finish(c, np, 2, S_DD_DOT);
    read_scalars(c, S_DD_DOT, 2);
    *action = c.hscal[S_DD_DOT];
    if (!(ok1 && ok2)) return DWF_ENOCONV;
    DWF_API_END
}

// ------------------------------------------------------- Chebyshev filter
//
// w_k = T_k(x(A)) v for A = Mpc^+ Mpc and x(A) = (2 A - (hi + lo)) / (hi - lo):
// w_0 = v, w_1 = x(A) v, w_{k+1} = 2 x(A) w_k - w_{k-1}.  Three fields rotate
// through the recurrence; each step is one A application (four stencil
// launches) and one three-term combination.

extern "C" dwf_status dwf_chebyshev_filter(dwf_ctx ctx, int prec, const double *v_odd, double lo, double hi,
                                           int nout, const int *orders, double *const *out_odd)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (prec < 0 || prec > 3) fail(DWF_EINVAL, "unknown precision");
    if (!v_odd || !orders || !out_odd) fail(DWF_EINVAL, "null pointer");
    if (nout < 1 || nout > 64) fail(DWF_EINVAL, "need 1 <= nout <= 64");
    if (!(std::isfinite(lo) && std::isfinite(hi) && lo >= 0.0 && hi > lo))
        fail(DWF_EINVAL, "need finite 0 <= lo < hi");
    for (int i = 0; i < nout; i++) {
        if (!out_odd[i]) fail(DWF_EINVAL, "null output pointer");
        if (orders[i] < 0 || orders[i] > 100000) fail(DWF_EINVAL, "orders must be in [0, 100000]");
        if (i > 0 && orders[i] <= orders[i - 1]) fail(DWF_EINVAL, "orders must be strictly ascending");
    }
    dwf::Context &c = *ctx;
    const int lp = prec;
    const double a = 2.0 / (hi - lo), sh = -(hi + lo) / (hi - lo);  // x(A) = a A + sh
    Field v64 = ws_field(c, "io_a", P_F64), e64 = ws_field(c, "io_b", P_F64);
    Field w[3] = {ws_field(c, "ch_w0", lp), ws_field(c, "ch_w1", lp), ws_field(c, "ch_w2", lp)};
    Field m = ws_field(c, "ch_m", lp), aw = ws_field(c, "ch_aw", lp);
    launch_import(c, P_F64, v_odd, v64, 0, 0);
    if (lp == P_F64) launch_copy(c, P_F64, v64, w[0]);
    else launch_convert(c, P_F64, v64, lp, w[0]);
    int next = 0;
    auto emit = [&](int k, Field f) {
        while (next < nout && orders[next] == k) {
            if (lp == P_F64) {
                launch_export(c, P_F64, f, out_odd[next], 0, 0);
            } else {
                launch_convert(c, lp, f, P_F64, e64);
                launch_export(c, P_F64, e64, out_odd[next], 0, 0);
            }
            next++;
        }
    };
    auto apply_a = [&](Field f) {
        apply_mpc(c, lp, false, f, m, false);
        apply_mpc(c, lp, true, m, aw, false);
    };
    emit(0, w[0]);
    const int kmax = orders[nout - 1];
    if (kmax >= 1) {
        apply_a(w[0]);
        launch_axpby(c, lp, a, aw, sh, w[0], w[1]);
        emit(1, w[1]);
    }
    for (int k = 2; k <= kmax; k++) {
        Field &wm = w[(k - 2) % 3], &w0 = w[(k - 1) % 3], &wn = w[k % 3];
        apply_a(w0);
        launch_axpbypcz(c, lp, 2.0 * a, aw, 2.0 * sh, w0, -1.0, wm, wn);
        emit(k, wn);
    }
    DWF_API_END
}
