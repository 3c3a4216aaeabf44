// Domain-boundary operators of the two-flavour boundary action (Sec. 2.1,
// the construction after eq. (schur)).
//
// The lattice splits into a domain Omega and its complement Omega-bar by a site
// mask.  Ordered by domain, D = [[D_Omega, D_d], [D_dbar, D_Omegabar]]; the cut
// operator D_cut = diag(D_Omega, D_Omegabar) is D5 on the gauge field whose
// links between the domains are zero (dwf_mask_links), held by a second
// context, and D_d + D_dbar = D - D_cut.  The projector P keeps the components
// of a field on Omega that D_dbar acts on, D_dbar P = D_dbar.  With
// D5 = Mooee - (1/2) H A the boundary hop sees (1 +- gamma_mu) A psi at a site
// of Omega next to Omega-bar, so P = A^-1 Pi A with Pi the spin-space mask of
// the boundary sites (an oblique projector for c != 0, the orthogonal spin
// mask for Shamir).  Then
//     R psi    = P psi - P D_Omega^-1 D_d D_Omegabar^-1 D_dbar psi,
//     R^-1 psi = P psi - P D^-1 D_dbar psi,
// with R R^-1 = P, and det R on the range of P equals the boundary
// determinant det chi, chi = 1 - D_Omega^-1 D_d D_Omegabar^-1 D_dbar.  The
// paper calls this part of the code performance non-critical; it composes
// the library's operator kernels and solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "dwf_internal.h"

namespace dwf {

// (D5 x) on both parities: Mooee x_p - (1/2) H_{p,1-p} A x_{1-p}, FP64 internal
static void d5_apply(Context &c, const Field x[2], const Field out[2])
{
    Field ax = ws_field(c, "bd_ax", P_F64);
    for (int par = 0; par < 2; par++) {
        launch_slocal(c, P_F64, SL_A, x[1 - par], ax);
        StencilSpec d5;
        d5.out_parity = par;
        d5.self = true;
        d5.s0 = c.d;
        d5.s1 = c.e;
        d5.tau = -0.5;
        launch_stencil(c, P_F64, d5, ax, x[par], out[par]);
    }
}

// out = P in = A^-1 Pi A in on both parities (in and out may alias)
static void project(Context &c, const int8_t *mask, const Field in[2], const Field out[2])
{
    Field t = ws_field(c, "bd_pt", P_F64);
    for (int par = 0; par < 2; par++) {
        launch_slocal(c, P_F64, SL_A, in[par], t);
        launch_boundary_mask(c, mask, t, t, par, 0);
        launch_slocal(c, P_F64, SL_AINV, t, out[par]);
    }
}

static void import_full(Context &c, const double *canon, const Field f[2])
{
    launch_import(c, P_F64, canon, f[0], 1, 0);
    launch_import(c, P_F64, canon, f[1], 1, 1);
}

static void export_full(Context &c, const Field f[2], double *canon)
{
    launch_export(c, P_F64, f[0], canon, 1, 0);
    launch_export(c, P_F64, f[1], canon, 1, 1);
}

static void pair(Context &c, const char *name, Field f[2])
{
    f[0] = ws_field(c, std::string(name) + "0", P_F64);
    f[1] = ws_field(c, std::string(name) + "1", P_F64);
}

// The mask is copied to the host once per call and checked: 0 or 1 on every
// site, both domains present.
static void check_mask(Context &c, const int8_t *mask)
{
    if (!mask) fail(DWF_EINVAL, "null mask");
    const long V = 2 * c.vh;
    std::vector<int8_t> h(V);
    HIPCHECK(hipMemcpyAsync(h.data(), mask, V, hipMemcpyDeviceToHost, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
    long ones = 0;
    for (int8_t m : h) {
        if (m != 0 && m != 1) fail(DWF_EINVAL, "mask entries must be 0 or 1");
        ones += m;
    }
    if (ones == 0 || ones == V) fail(DWF_EINVAL, "the mask must mark a proper, non-empty domain");
}

static void check_boundary_params(const Context &c)
{
    if (c.p.b == 0.0) fail(DWF_ENOTSUP, "the boundary projector needs A = b + c P5 with b != 0");
    const double g = -c.p.c / c.p.b;
    if (std::fabs(1.0 + c.p.mf * std::pow(g, c.Ls)) < 1e-12) fail(DWF_ENOTSUP, "A = b + c P5 is singular");
}

static void check_same_lattice(const Context &a, const Context &b)
{
    bool same = a.Ls == b.Ls && a.p.b == b.p.b && a.p.c == b.p.c && a.p.M5 == b.p.M5 && a.p.mf == b.p.mf;
    for (int mu = 0; mu < 4; mu++) same = same && a.L[mu] == b.L[mu];
    if (!same) fail(DWF_EINVAL, "the cut context must have the lattice and parameters of the full one");
}

}  // namespace dwf

using namespace dwf;

extern "C" dwf_status dwf_mask_links(dwf_ctx ctx, const int8_t *mask, const double *gauge_in, double *gauge_out)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!gauge_in || !gauge_out) fail(DWF_EINVAL, "null gauge pointer");
    Context &c = *ctx;
    check_mask(c, mask);
    launch_mask_links(c, mask, gauge_in, gauge_out);
    HIPCHECK(hipStreamSynchronize(c.stream));
    DWF_API_END
}

extern "C" dwf_status dwf_d5_apply(dwf_ctx ctx, const double *in_full, double *out_full)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!in_full || !out_full) fail(DWF_EINVAL, "null field pointer");
    Context &c = *ctx;
    Field x[2], y[2];
    pair(c, "bd_x", x);
    pair(c, "bd_y", y);
    import_full(c, in_full, x);
    d5_apply(c, x, y);
    export_full(c, y, out_full);
    DWF_API_END
}

extern "C" dwf_status dwf_boundary_project(dwf_ctx ctx, const int8_t *mask, const double *in_full, double *out_full)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!in_full || !out_full) fail(DWF_EINVAL, "null field pointer");
    Context &c = *ctx;
    check_mask(c, mask);
    check_boundary_params(c);
    Field x[2];
    pair(c, "bd_x", x);
    import_full(c, in_full, x);
    project(c, mask, x, x);
    export_full(c, x, out_full);
    DWF_API_END
}

extern "C" dwf_status dwf_boundary_apply(dwf_ctx ctx, dwf_ctx ctx_cut, const int8_t *mask, int inverse,
                                         const double *in_full, double *out_full, const dwf_solver_opts *o,
                                         dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx || !ctx_cut) fail(DWF_EINVAL, "null context");
    if (ctx == ctx_cut) fail(DWF_EINVAL, "the cut context must be a second context");
    if (!in_full || !out_full) fail(DWF_EINVAL, "null field pointer");
    if (inverse != 0 && inverse != 1) fail(DWF_EINVAL, "inverse must be 0 or 1");
    Context &c = *ctx;
    Context &cc = *ctx_cut;
    check_same_lattice(c, cc);
    check_mask(c, mask);
    check_boundary_params(c);
    dwf_solver_opts so = o ? *o : dwf_solver_opts{};
    so.x0_is_guess = 0;
    const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    // canonical full fields for the cut context and the solves, internal FP64
    // fields of the full context for everything else
    const size_t cbytes = (size_t)2 * c.n5h * 12 * 2 * sizeof(double);
    double *can0 = (double *)ws_raw(c, "bd_can0", cbytes);
    double *can1 = (double *)ws_raw(c, "bd_can1", cbytes);
    Field x[2], y[2], z[2];
    pair(c, "bd_x", x);
    pair(c, "bd_y", y);
    pair(c, "bd_z", z);
    dwf_solver_stats total{};
    total.converged = 1;
    auto solve = [&](dwf_ctx on, const double *b, double *xs) {
        dwf_solver_stats s{};
        HIPCHECK(hipStreamSynchronize(c.stream));
        const dwf_status r = dwf_cg(on, b, xs, &so, &s);
        if (r != DWF_OK && r != DWF_ENOCONV) fail(r, std::string("boundary solve: ") + dwf_last_error());
        HIPCHECK(hipStreamSynchronize(on->stream));
        total.iters += s.iters;
        total.reliable_updates += s.reliable_updates;
        total.converged = total.converged && s.converged;
        total.res_full = std::max(total.res_full, s.res_full);
        total.res_normal = std::max(total.res_normal, s.res_normal);
        total.res_schur = std::max(total.res_schur, s.res_schur);
        total.t_solve += s.seconds;
    };
    // u = (D - D_cut) v for v on one domain (internal in v, canonical copy in
    // can0), into the internal fields y; z is used as scratch
    auto boundary_hop = [&](const Field v[2]) {
        export_full(c, v, can0);
        HIPCHECK(hipStreamSynchronize(c.stream));
        const dwf_status r = dwf_d5_apply(ctx_cut, can0, can1);
        if (r != DWF_OK) fail(r, std::string("cut operator: ") + dwf_last_error());
        HIPCHECK(hipStreamSynchronize(cc.stream));
        d5_apply(c, v, y);
        import_full(c, can1, z);
        for (int par = 0; par < 2; par++) launch_axpby(c, P_F64, 1.0, y[par], -1.0, z[par], y[par]);
    };
    // psi on Omega
    import_full(c, in_full, x);
    for (int par = 0; par < 2; par++) launch_boundary_mask(c, mask, x[par], x[par], par, 1);
    boundary_hop(x);  // y = D_dbar psi, on Omega-bar
    export_full(c, y, can0);
    if (inverse) {
        solve(ctx, can0, can1);  // D^-1 D_dbar psi
    } else {
        solve(ctx_cut, can0, can1);  // D_Omegabar^-1 D_dbar psi
        import_full(c, can1, x);
        boundary_hop(x);  // y = D_d D_Omegabar^-1 D_dbar psi, on Omega
        export_full(c, y, can0);
        solve(ctx_cut, can0, can1);  // D_Omega^-1 ...
    }
    import_full(c, can1, z);
    project(c, mask, z, z);
    import_full(c, in_full, x);
    for (int par = 0; par < 2; par++) launch_boundary_mask(c, mask, x[par], x[par], par, 1);
    project(c, mask, x, x);
    for (int par = 0; par < 2; par++) launch_axpby(c, P_F64, 1.0, x[par], -1.0, z[par], x[par]);
    export_full(c, x, out_full);
    HIPCHECK(hipStreamSynchronize(c.stream));
    if (st) {
        *st = total;
        st->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
    }
    if (!total.converged) return DWF_ENOCONV;
    DWF_API_END
}
