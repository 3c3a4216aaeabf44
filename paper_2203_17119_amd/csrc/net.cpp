// Learned preconditioner: network lifecycle, forward / backward / training
// step on the device, the preconditioner application and flexible GCR.
//
// Weights: per layer l a block W_l[pi][a][b] of 11 x Cout x Cin complex
// numbers, layers back to back.  The host-facing format is FP32 (re, im)
// pairs; the device keeps FP32 masters (Adam) and the BF16 copies the kernels
// use.  Gradients follow the real-pair convention dL/dRe + i dL/dIm.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "dwf_internal.h"

using namespace dwf;

namespace dwf {
// pmask: the paths (bit pi) to evaluate; the others must have zero sources
constexpr int kAllPaths = 0x7ff;
void launch_ptc_layer(Context &c, int cin, int cout, const float2 *in, float2 *out, const void *w_bf16, int p,
                      int pmask = kAllPaths);
size_t mfma_weight_elems(int cin);
void launch_pack_mfma_weights(Context &c, int cin, int cout, const void *w_bf16, short *pk);
void launch_ptc_layer_mfma(Context &c, int cin, int cout, const void *in, void *out, const short *pk, int p,
                           bool in_bf16, bool out_bf16, int pmask = kAllPaths, int io = 0);
int launch_ptc_wgrad(Context &c, int cin, int cout, const float2 *in, const float2 *gout, int p, double *partial,
                     long partial_len);
void launch_wgrad_finish(Context &c, const double *partial, int nblk, int nw, float *gw, bool accumulate);
void launch_adjoint_weights(Context &c, const void *w, void *wt, int cin, int cout);
void launch_to_bf16(Context &c, const float *w, void *o, int nw);
void launch_adam(Context &c, float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                 float eps, int step);
void launch_spinor_to_feat(Context &c, int prec, Field f, float2 *feat, int p, bool zero_other);
void launch_feat_to_spinor(Context &c, int prec, const float2 *feat, Field f, int p);
int launch_loss_residual(Context &c, const float2 *y, Field x, float2 *grad, int p);
void launch_scale_feat(Context &c, float2 *f, long n, float a);
void launch_zero_feat(Context &c, float2 *f, long n);
}  // namespace dwf

struct dwf_net_s {
    Context *c = nullptr;
    int nlayer = 0;
    std::vector<int> chans;
    std::vector<int> woff;  // complex offset of each layer's block
    int nw = 0;             // complex weights in total
    float *w32 = nullptr, *gw = nullptr, *m = nullptr, *v = nullptr;
    void *wbf = nullptr, *wadj = nullptr;
    int step = 0;
    std::vector<float2 *> acts;  // layer inputs (both parities), acts[nlayer] = output
    std::vector<void *> acts_bf;  // BF16 inputs of layers 1 .. nlayer-1 for the matrix-core forward
    float2 *g0 = nullptr, *g1 = nullptr;  // gradient ping-pong (max channels)
    double *wpart = nullptr;
    long wpart_len = 0;
    int cmax = 0;
    short *wpk = nullptr;          // matrix-core operand order, per layer at pkoff[l]
    std::vector<size_t> pkoff;
    int fwd = DWF_NET_FWD_FP32;    // forward used by the preconditioner application
};

namespace dwf {

static double wall()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static size_t feat_elems(const Context &c, int C) { return (size_t)2 * C * 3 * c.n5h; }

static void net_free(dwf_net_s *n)
{
    for (void *p : {(void *)n->w32, (void *)n->gw, (void *)n->m, (void *)n->v, n->wbf, n->wadj, (void *)n->g0,
                    (void *)n->g1, (void *)n->wpart, (void *)n->wpk})
        if (p) (void)hipFree(p);
    for (auto *a : n->acts)
        if (a) (void)hipFree(a);
    for (auto *a : n->acts_bf)
        if (a) (void)hipFree(a);
    delete n;
}

static void refresh_bf16(dwf_net_s *n)
{
    Context &c = *n->c;
    launch_to_bf16(c, n->w32, n->wbf, n->nw);
    for (int l = 0; l < n->nlayer; l++) {
        launch_adjoint_weights(c, (const __hip_bfloat162 *)n->wbf + n->woff[l], (__hip_bfloat162 *)n->wadj + n->woff[l],
                               n->chans[l], n->chans[l + 1]);
        launch_pack_mfma_weights(c, n->chans[l], n->chans[l + 1], (const __hip_bfloat162 *)n->wbf + n->woff[l],
                                 n->wpk + n->pkoff[l]);
    }
}

// forward of one sample whose input is acts[0] (4 channels); the last layer
// is evaluated on odd sites only (the preconditioner's range)
// (mfma: the matrix-core forward, BF16 operands with FP32 accumulation)
// The network input is an odd-site field embedded with zeros on the even
// sites, so the first layer skips the paths that only read even sites: for the
// odd output the eight hops (they come from the other parity), for the even
// output the identity and s-paths.  The forward therefore never reads the even
// part of acts[0]; the callers that run the adjoint or train clear it.
static constexpr int kHopPaths = 0x1fe, kLocalPaths = 0x601;

// With the matrix-core forward the first layer may read the odd half spinor
// in_sp (FP32 or BF16, in_prec) instead of acts[0], and the last layer (odd
// sites only) may write the odd half spinor out_sp (FP32 or BF16, out_prec)
// instead of acts[nlayer]: the layout conversions then cost no pass of their own.
static void net_forward(dwf_net_s *n, bool all_parities, bool mfma = false, Field in_sp = {}, Field out_sp = {},
                        int out_prec = P_F32, int in_prec = P_F32)
{
    Context &c = *n->c;
    for (int l = 0; l < n->nlayer; l++) {
        const bool last = l == n->nlayer - 1;
        for (int p = (last && !all_parities) ? 1 : 0; p < 2; p++) {
            const int pmask = l > 0 ? kAllPaths : (p == 1 ? kLocalPaths : kHopPaths);
            if (mfma) {
                // FP32 (or BF16 spinor) network input, FP32 output, BF16 activations in between
                const bool isp = l == 0 && in_sp.data, osp = last && out_sp.data && !all_parities;
                const bool ibf = l > 0 || (isp && in_prec == P_BF16), obf = !last;
                const int io = (isp ? 1 : 0) | (osp ? (out_prec == P_BF16 ? 4 : 2) : 0);
                const void *src = isp ? in_sp.data : ibf ? n->acts_bf[l] : (const void *)n->acts[l];
                void *dst = osp ? out_sp.data : obf ? n->acts_bf[l + 1] : (void *)n->acts[l + 1];
                launch_ptc_layer_mfma(c, n->chans[l], n->chans[l + 1], src, dst, n->wpk + n->pkoff[l], p, ibf, obf,
                                      pmask, io);
            } else {
                launch_ptc_layer(c, n->chans[l], n->chans[l + 1], n->acts[l], n->acts[l + 1],
                                 (const __hip_bfloat162 *)n->wbf + n->woff[l], p, pmask);
            }
        }
    }
}

// adjoint network applied to features g (4 channels, both parities, not g0/g1);
// returns the buffer (g0 or g1) holding the 4-channel result
static float2 *net_adjoint(dwf_net_s *n, const float2 *g)
{
    Context &c = *n->c;
    const float2 *cur = g;
    float2 *dst = nullptr;
    for (int l = n->nlayer - 1; l >= 0; l--) {
        dst = (cur == n->g0) ? n->g1 : n->g0;
        for (int p = 0; p < 2; p++)
            launch_ptc_layer(c, n->chans[l + 1], n->chans[l], cur, dst, (const __hip_bfloat162 *)n->wadj + n->woff[l], p);
        cur = dst;
    }
    return dst;
}

// backward from the gradient in g0 (4 output channels, both parities, even part
// zero): accumulates the weight gradient into gw and leaves the input gradient in
// the returned buffer
static float2 *net_backward(dwf_net_s *n)
{
    Context &c = *n->c;
    float2 *g = n->g0, *o = n->g1;
    for (int l = n->nlayer - 1; l >= 0; l--) {
        const int cin = n->chans[l], cout = n->chans[l + 1];
        const int nwl = 11 * cin * cout;
        for (int p = (l == n->nlayer - 1) ? 1 : 0; p < 2; p++) {
            const int nb = launch_ptc_wgrad(c, cin, cout, n->acts[l], g, p, n->wpart, n->wpart_len);
            launch_wgrad_finish(c, n->wpart, nb, nwl, n->gw + 2 * (size_t)n->woff[l], true);
        }
        for (int p = 0; p < 2; p++)
            launch_ptc_layer(c, cout, cin, g, o, (const __hip_bfloat162 *)n->wadj + n->woff[l], p);
        std::swap(g, o);
    }
    return g;
}

}  // namespace dwf

// ================================================================ C ABI

static dwf_net_s &N_(dwf_net n)
{
    if (!n) fail(DWF_EINVAL, "null network");
    return *n;
}

extern "C" {

dwf_status dwf_net_create(dwf_ctx ctx, int nlayer, const int *chans, dwf_net *out)
{
    DWF_API_BEGIN
    if (!ctx || !chans || !out) fail(DWF_EINVAL, "null pointer");
    *out = nullptr;
    if (nlayer < 1 || nlayer > 16) fail(DWF_EINVAL, "1 <= nlayer <= 16");
    if (chans[0] != 4 || chans[nlayer] != 4) fail(DWF_EINVAL, "the first and last channel counts must be 4 (spins)");
    for (int l = 0; l <= nlayer; l++)
        if (chans[l] != 4 && chans[l] != 8 && chans[l] != 12) fail(DWF_ENOTSUP, "channel counts must be 4, 8 or 12");
    Context &c = *ctx;
    auto *n = new dwf_net_s();
    try {
        n->c = &c;
        n->nlayer = nlayer;
        n->chans.assign(chans, chans + nlayer + 1);
        for (int l = 0; l < nlayer; l++) {
            n->woff.push_back(n->nw);
            n->nw += 11 * chans[l] * chans[l + 1];
        }
        for (int ch : n->chans) n->cmax = std::max(n->cmax, ch);
        ensure_links(c, P_F32);
        HIPCHECK(hipMalloc(&n->w32, 2 * sizeof(float) * n->nw));
        HIPCHECK(hipMalloc(&n->gw, 2 * sizeof(float) * n->nw));
        HIPCHECK(hipMalloc(&n->m, 2 * sizeof(float) * n->nw));
        HIPCHECK(hipMalloc(&n->v, 2 * sizeof(float) * n->nw));
        HIPCHECK(hipMalloc(&n->wbf, 4 * (size_t)n->nw));
        size_t pk = 0;
        for (int l = 0; l < nlayer; l++) {
            n->pkoff.push_back(pk);
            pk += mfma_weight_elems(chans[l]);
        }
        HIPCHECK(hipMalloc(&n->wpk, pk * sizeof(short)));
        HIPCHECK(hipMalloc(&n->wadj, 4 * (size_t)n->nw));
        for (void *p : {(void *)n->w32, (void *)n->gw, (void *)n->m, (void *)n->v})
            HIPCHECK(hipMemset(p, 0, 2 * sizeof(float) * n->nw));
        for (int l = 0; l <= nlayer; l++) {
            float2 *a = nullptr;
            HIPCHECK(hipMalloc(&a, feat_elems(c, chans[l]) * sizeof(float2)));
            n->acts.push_back(a);
            void *b = nullptr;
            if (l > 0 && l < nlayer) HIPCHECK(hipMalloc(&b, feat_elems(c, chans[l]) * sizeof(__hip_bfloat162)));
            n->acts_bf.push_back(b);
        }
        HIPCHECK(hipMalloc(&n->g0, feat_elems(c, n->cmax) * sizeof(float2)));
        HIPCHECK(hipMalloc(&n->g1, feat_elems(c, n->cmax) * sizeof(float2)));
        const int sbn = std::max(1, std::min(64, 128 / c.Ls));
        const long nblk = (c.vh + sbn - 1) / sbn;
        n->wpart_len = nblk * 11 * (long)n->cmax * n->cmax * 2;
        HIPCHECK(hipMalloc(&n->wpart, n->wpart_len * sizeof(double)));
        refresh_bf16(n);
        HIPCHECK(hipStreamSynchronize(c.stream));
    } catch (...) {
        net_free(n);
        throw;
    }
    *out = n;
    DWF_API_END
}

dwf_status dwf_net_destroy(dwf_net net)
{
    if (!net) return DWF_OK;
    (void)hipStreamSynchronize(net->c->stream);
    net_free(net);
    return DWF_OK;
}

int dwf_net_num_weights(dwf_net net) { return net ? net->nw : -1; }

dwf_status dwf_net_set_weights(dwf_net net, const float *w)
{
    DWF_API_BEGIN
    dwf_net_s &n = N_(net);
    if (!w) fail(DWF_EINVAL, "null weights");
    HIPCHECK(hipMemcpy(n.w32, w, 2 * sizeof(float) * n.nw, hipMemcpyHostToDevice));
    HIPCHECK(hipMemset(n.m, 0, 2 * sizeof(float) * n.nw));
    HIPCHECK(hipMemset(n.v, 0, 2 * sizeof(float) * n.nw));
    n.step = 0;
    refresh_bf16(&n);
    HIPCHECK(hipStreamSynchronize(n.c->stream));
    DWF_API_END
}

dwf_status dwf_net_get_weights(dwf_net net, float *w)
{
    DWF_API_BEGIN
    dwf_net_s &n = N_(net);
    if (!w) fail(DWF_EINVAL, "null weights");
    HIPCHECK(hipStreamSynchronize(n.c->stream));
    HIPCHECK(hipMemcpy(w, n.w32, 2 * sizeof(float) * n.nw, hipMemcpyDeviceToHost));
    DWF_API_END
}

dwf_status dwf_net_set_forward(dwf_net net, int mode)
{
    DWF_API_BEGIN
    dwf_net_s &n = N_(net);
    if (mode != DWF_NET_FWD_FP32 && mode != DWF_NET_FWD_MFMA_BF16) fail(DWF_EINVAL, "unknown forward mode");
    n.fwd = mode;
    DWF_API_END
}

dwf_status dwf_precond_apply(dwf_ctx ctx, dwf_net net, const double *in_odd, double *out_odd)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    dwf_net_s &n = N_(net);
    if (n.c != ctx) fail(DWF_EINVAL, "network belongs to another context");
    if (!in_odd || !out_odd) fail(DWF_EINVAL, "null field");
    Context &c = *ctx;
    Field a = ws_field(c, "net_io", P_F64);
    launch_import(c, P_F64, in_odd, a, 0, 0);
    launch_spinor_to_feat(c, P_F64, a, n.acts[0], 1, true);
    net_forward(&n, false, n.fwd == DWF_NET_FWD_MFMA_BF16);
    launch_feat_to_spinor(c, P_F64, n.acts[n.nlayer], a, 1);
    launch_export(c, P_F64, a, out_odd, 0, 0);
    DWF_API_END
}

dwf_status dwf_net_backward(dwf_net net, const double *in_odd, const double *grad_out_odd, double *grad_in_odd,
                            float *grad_w)
{
    DWF_API_BEGIN
    dwf_net_s &n = N_(net);
    if (!in_odd || !grad_out_odd) fail(DWF_EINVAL, "null field");
    Context &c = *n.c;
    Field a = ws_field(c, "net_io", P_F64);
    launch_import(c, P_F64, in_odd, a, 0, 0);
    launch_spinor_to_feat(c, P_F64, a, n.acts[0], 1, true);
    net_forward(&n, false);
    launch_import(c, P_F64, grad_out_odd, a, 0, 0);
    launch_spinor_to_feat(c, P_F64, a, n.g0, 1, true);
    HIPCHECK(hipMemsetAsync(n.gw, 0, 2 * sizeof(float) * n.nw, c.stream));
    float2 *gin = net_backward(&n);
    if (grad_in_odd) {
        launch_feat_to_spinor(c, P_F64, gin, a, 1);
        launch_export(c, P_F64, a, grad_in_odd, 0, 0);
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    if (grad_w) HIPCHECK(hipMemcpy(grad_w, n.gw, 2 * sizeof(float) * n.nw, hipMemcpyDeviceToHost));
    DWF_API_END
}

dwf_status dwf_net_train_step(dwf_net net, int nbatch, const double *const *b_odd, const double *const *x_odd,
                              const dwf_adam *opt, double *loss)
{
    DWF_API_BEGIN
    dwf_net_s &n = N_(net);
    if (nbatch < 1 || !b_odd || !x_odd) fail(DWF_EINVAL, "need nbatch >= 1 and field arrays");
    Context &c = *n.c;
    Field a = ws_field(c, "net_io", P_F64), xt = ws_field(c, "net_x", P_F64);
    HIPCHECK(hipMemsetAsync(n.gw, 0, 2 * sizeof(float) * n.nw, c.stream));
    double total = 0;
    for (int k = 0; k < nbatch; k++) {
        if (!b_odd[k] || !x_odd[k]) fail(DWF_EINVAL, "null field in batch");
        launch_import(c, P_F64, b_odd[k], a, 0, 0);
        launch_import(c, P_F64, x_odd[k], xt, 0, 0);
        launch_spinor_to_feat(c, P_F64, a, n.acts[0], 1, true);
        net_forward(&n, false);
        // loss_k = |y - x|^2 / |x|^2 on odd sites; gradient 2 (y - x) / (|x|^2 B)
        launch_zero_feat(c, n.g0, (long)2 * 12 * c.n5h);
        const int nb = launch_loss_residual(c, n.acts[n.nlayer], xt, n.g0, 1);
        launch_finish(c, nb, 2, 10);
        read_scalars(c, 10, 2);
        const double r2 = c.hscal[10], x2 = c.hscal[11];
        if (!(x2 > 0)) fail(DWF_EINVAL, "zero target field");
        total += r2 / x2;
        launch_scale_feat(c, n.g0 + 12 * c.n5h, 12 * c.n5h, (float)(2.0 / (x2 * nbatch)));
        net_backward(&n);
    }
    if (loss) *loss = total / nbatch;
    if (opt) {
        n.step++;
        launch_adam(c, n.w32, n.gw, n.m, n.v, 2 * n.nw, (float)opt->lr, (float)opt->beta1, (float)opt->beta2,
                    (float)opt->eps, n.step);
        refresh_bf16(&n);
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    DWF_API_END
}

}  // extern "C"

// ---------------------------------------------------------------- FGCR

namespace dwf {

// z = N(r) (normal = false) or N N^+ r (normal = true), odd fields of precision prec
// z = N r (N N^+ r for the normal equations); r is read in precision rprec, z
// is written in zprec
static void precondition(dwf_net_s *n, int rprec, Field r, int zprec, Field z, bool normal)
{
    Context &c = *n->c;
    const bool mfma = n->fwd == DWF_NET_FWD_MFMA_BF16;
    // (a BF16 input spinor feeds a first layer that writes BF16 activations:
    // a network of one layer takes the feature path)
    const bool rsp = rprec == P_F32 || (rprec == P_BF16 && n->nlayer >= 2);
    if (!normal && mfma && rsp && (zprec == P_F32 || zprec == P_BF16)) {
        // the first layer reads r and the last writes z in their spinor layouts
        net_forward(n, false, true, r, z, zprec, rprec);
        return;
    }
    // the forward alone reads only the odd sites of its input (the first
    // layer's path mask), so the even part need not be cleared; the adjoint
    // reads both parities
    launch_spinor_to_feat(c, rprec, r, n->acts[0], 1, normal);
    if (normal) {
        // N^+ r: adjoint network on the embedded residual, then N on its result
        const float2 *adj = net_adjoint(n, n->acts[0]);
        launch_feat_to_spinor(c, zprec, adj, z, 1);  // keep odd part only
        launch_spinor_to_feat(c, zprec, z, n->acts[0], 1, true);
    }
    net_forward(n, false, mfma);
    launch_feat_to_spinor(c, zprec, n->acts[n->nlayer], z, 1);
}

static double dnorm2(Context &c, Field a)
{
    const int np = launch_norm2(c, P_F64, a);
    launch_finish(c, np, 1, 12);
    read_scalars(c, 12, 1);
    return c.hscal[12];
}

static void ddot(Context &c, Field a, Field b, double &re, double &im)
{
    const int np = launch_dot(c, P_F64, a, b);
    launch_finish(c, np, 2, 14);
    read_scalars(c, 14, 2);
    re = c.hscal[14];
    im = c.hscal[15];
}

static void fgcr_op(Context &c, int prec, Field in, Field out, bool normal)
{
    if (normal) {
        Field t = ws_field(c, "fg_t", prec);
        apply_mpc(c, prec, false, in, t, false);
        apply_mpc(c, prec, true, t, out, false);
    } else {
        apply_mpc(c, prec, false, in, out, false);
    }
}

}  // namespace dwf

extern "C" dwf_status dwf_precond_apply_internal(dwf_ctx ctx, dwf_net net, int in_prec, const void *in, int out_prec,
                                                 void *out)
{
    DWF_API_BEGIN
    if (!ctx || !net) fail(DWF_EINVAL, "null context or network");
    if (net->c != ctx) fail(DWF_EINVAL, "network belongs to another context");
    if (!in || !out) fail(DWF_EINVAL, "null field");
    if (in_prec < P_F64 || in_prec > P_BF16 || out_prec < P_F64 || out_prec > P_BF16)
        fail(DWF_EINVAL, "unknown precision");
    if (in == out) fail(DWF_EINVAL, "in and out must differ");
    Context &c = *ctx;
    precondition(net, in_prec, make_field(c, (void *)in, in_prec), out_prec, make_field(c, out, out_prec), false);
    DWF_API_END
}

extern "C" dwf_status dwf_fgcr(dwf_ctx ctx, dwf_net net, const double *b_full, double *x_full,
                               const dwf_solver_opts *o, dwf_solver_stats *st)
{
    DWF_API_BEGIN
    if (!ctx || !b_full || !x_full) fail(DWF_EINVAL, "null pointer");
    Context &c = *ctx;
    if (net && net->c != ctx) fail(DWF_EINVAL, "network belongs to another context");
    const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
    const int maxit = (o && o->maxit > 0) ? o->maxit : 20000;
    const int m = (o && o->restart > 0) ? std::min(o->restart, 64) : 16;
    const bool normal = o && o->normal;
    const bool fallback = !o || o->fallback;
    // inner precision: FP64; or FP32 vectors and operator with the solution and
    // the residual of every restart kept in FP64 (reliable restarts); or, for
    // MIXED_BF16, the same with the Krylov basis (the preconditioned directions
    // and their images) stored in BF16 and the operator applied in BF16 storage,
    // while the cycle's residual and solution stay FP32
    const int mode = o ? o->mode : DWF_SOLVE_F64;
    if (mode != DWF_SOLVE_F64 && mode != DWF_SOLVE_MIXED_F32 && mode != DWF_SOLVE_MIXED_BF16)
        fail(DWF_ENOTSUP, "FGCR mode must be F64, MIXED_F32 or MIXED_BF16");
    const int lp = mode == DWF_SOLVE_MIXED_F32 ? P_F32 : mode == DWF_SOLVE_MIXED_BF16 ? P_BF16 : P_F64;
    const int rp = lp == P_BF16 ? P_F32 : lp;  // residual and solution of a cycle
    const bool mixed = lp != P_F64;
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t0 = wall();
    Field be = ws_field(c, "sv_be", P_F64), bo = ws_field(c, "sv_bo", P_F64), bt = ws_field(c, "sv_bt", P_F64);
    Field rhs = ws_field(c, "fg_rhs", P_F64), x = ws_field(c, "sv_xo", P_F64), r = ws_field(c, "fg_r", P_F64);
    Field t1 = ws_field(c, "sv_t1", P_F64);
    launch_import(c, P_F64, b_full, be, 1, 0);
    launch_import(c, P_F64, b_full, bo, 1, 1);
    launch_slocal(c, P_F64, SL_E1, be, t1);
    StencilSpec sp;
    sp.out_parity = 1;
    sp.self = true;
    sp.s0 = 1.0;
    sp.tau = 0.5;
    launch_stencil(c, P_F64, sp, t1, bo, bt);
    if (normal) apply_mpc(c, P_F64, true, bt, rhs, false);
    else launch_copy(c, P_F64, bt, rhs);
    std::vector<Field> Z, Q;
    for (int k = 0; k < m; k++) {
        Z.push_back(ws_field(c, "fg_z" + std::to_string(k), lp));
        Q.push_back(ws_field(c, "fg_q" + std::to_string(k), lp));
    }
    Field rl = mixed ? ws_field(c, "fg_rl", rp) : r, xl = mixed ? ws_field(c, "fg_xl", rp) : x;
    // With a BF16 basis and the matrix-core forward the network reads a BF16
    // copy of the cycle's residual, written by the update kernel beside the
    // FP32 one: its first layer rounds its operands to BF16 anyway, and the
    // gathers of its first layer then move half the bytes.
    const bool rb_in = lp == P_BF16 && net && net->fwd == DWF_NET_FWD_MFMA_BF16 && !normal && net->nlayer >= 2;
    Field rb = rb_in ? ws_field(c, "fg_rb", P_BF16) : Field{};
    // device pointer tables of the Krylov vectors, Gram-Schmidt coefficients
    // (dots[2m] per step; info[3k] = {|q_k|^2, <q_k, r>} per step; cc[3m], the
    // combination coefficients of a BF16 cycle) and partial sums
    struct Dev {
        void *p = nullptr;
        ~Dev()
        {
            if (p) (void)hipFree(p);
        }
    } tab, coef, part;
    HIPCHECK(hipMalloc(&tab.p, 2 * m * sizeof(void *)));
    HIPCHECK(hipMalloc(&coef.p, (2 * m * m + 3 * m + 3 * m) * sizeof(double)));
    HIPCHECK(hipMalloc(&part.p, gs_partials_needed(c, m) * sizeof(double)));
    {
        std::vector<const void *> h(2 * m);
        for (int k = 0; k < m; k++) {
            h[k] = Q[k].data;
            h[m + k] = Z[k].data;
        }
        HIPCHECK(hipMemcpy(tab.p, h.data(), h.size() * sizeof(void *), hipMemcpyHostToDevice));
    }
    void *const *qtab = (void *const *)tab.p;
    void *const *ztab = qtab + m;
    double *dots = (double *)coef.p, *info = dots + 2 * m * m, *cc = info + 3 * m;
    double *partial = (double *)part.p;
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t1w = wall();
    const double bn = std::sqrt(dnorm2(c, rhs));
    launch_zero(c, P_F64, x);
    launch_copy(c, P_F64, rhs, r);
    if (mixed) launch_zero(c, rp, xl);
    int it = 0;
    bool conv = bn == 0.0, stalled = false;
    // stagnation is judged on the true residual of the restarts: no 10% gain
    // over many steps.  The cycle's own residual can run below the true one
    // when the basis is stored in BF16, and restarted GCR on a non-normal
    // operator has long plateaus of slow progress that are not stagnation.
    double best = bn;
    int best_it = 0;
    while (!conv && !stalled && it < maxit) {
        int k = 0, ndir = 0;  // ndir: directions of this cycle applied to the residual
        // With a BF16 basis the cycle's solution update is combined at the
        // restart, from the directions as the preconditioner made them: only
        // their operator images are projected, and the projection coefficients
        // of every step are kept to transform the combination (as flexible
        // GMRES keeps its raw directions).  That halves the Gram-Schmidt
        // traffic of the directions.
        const bool defer_x = lp == P_BF16;
        if (mixed) launch_convert(c, P_F64, r, rp, rl);
        if (rb_in) launch_convert(c, P_F64, r, P_BF16, rb);
        for (; k < m && it < maxit; k++) {
            if (rb_in) precondition(net, P_BF16, rb, lp, Z[k], normal);
            else if (net) precondition(net, rp, rl, lp, Z[k], normal);
            else if (rp == lp) launch_copy(c, lp, rl, Z[k]);
            else launch_convert(c, rp, rl, lp, Z[k]);
            fgcr_op(c, lp, Z[k], Q[k], normal);
            // classical Gram-Schmidt against the cycle's earlier directions in
            // one pass over the vectors; the residual stays orthogonal to them
            double *dk = defer_x ? dots + 2 * m * k : dots;
            if (k > 0) launch_gs_dots(c, lp, (const void *const *)qtab, k, Q[k], partial, dk);
            launch_gs_project(c, lp, rp, (const void *const *)qtab, defer_x ? nullptr : (const void *const *)ztab, k,
                              dk, info, Q[k], defer_x ? Field{} : Z[k], rl, partial, info + 3 * k);
            const int np = launch_gs_update(c, lp, rp, defer_x ? Field{} : xl, Z[k], rl, Q[k], info + 3 * k, rb);
            ndir = k + 1;
            launch_finish(c, np, 1, 12);
            read_scalars(c, 12, 1);
            it++;
            const double rn = std::sqrt(c.hscal[12]);
            if (!std::isfinite(rn)) {
                stalled = true;
                break;
            }
            if (rn <= tol * bn) break;
        }
        // restart: fold the low-precision solution in, true residual in FP64
        if (defer_x && ndir > 0) {
            launch_gs_raw_coef(c, ndir, 2 * m, dots, info, cc);
            launch_gs_combine(c, lp, xl, (const void *const *)ztab, ndir, cc);
        }
        if (mixed) launch_accumulate_low(c, rp, x, xl);
        fgcr_op(c, P_F64, x, t1, normal);
        launch_axpby(c, P_F64, 1.0, rhs, -1.0, t1, r);
        const double rn = std::sqrt(dnorm2(c, r));
        if (!std::isfinite(rn)) stalled = true;
        if (rn <= tol * bn) conv = true;
        if (rn < 0.9 * best) {
            best = rn;
            best_it = it;
        } else if (it - best_it > std::max(8 * m, 256)) {
            stalled = true;
        }
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t2w = wall();
    int fell = 0;
    dwf_status status = DWF_OK;
    if (!conv) {
        if (!fallback) {
            status = DWF_ENOCONV;
        } else {
            fell = 1;
        }
    }
    if (fell) {
        dwf_solver_opts co{};
        co.tol = tol;
        co.maxit = o && o->maxit > 0 ? o->maxit : 0;
        co.mode = DWF_SOLVE_F64;
        dwf_solver_stats cs{};
        status = dwf_cg(ctx, b_full, x_full, &co, &cs);
        if (st) {
            *st = cs;
            st->fell_back = 1;
            st->iters += it;
            st->seconds = wall() - t0;
        }
        return status;
    }
    // reconstruct, residuals (shared with the CG path's final stage)
    Field t2 = ws_field(c, "sv_t2", P_F64), xe = ws_field(c, "sv_xe", P_F64), ax = ws_field(c, "sv_ax", P_F64);
    launch_slocal(c, P_F64, SL_A, x, t1);
    sp = StencilSpec{};
    sp.out_parity = 0;
    sp.self = true;
    sp.s0 = 1.0;
    sp.tau = 0.5;
    launch_stencil(c, P_F64, sp, t1, be, t2);
    launch_slocal(c, P_F64, SL_MINV, t2, xe);
    launch_export(c, P_F64, xe, x_full, 1, 0);
    launch_export(c, P_F64, x, x_full, 1, 1);
    apply_mpc(c, P_F64, false, x, t1, false);
    launch_axpby(c, P_F64, 1.0, bt, -1.0, t1, t1);
    const double bt2 = dnorm2(c, bt), rs2 = dnorm2(c, t1);
    apply_mpc(c, P_F64, true, t1, t2, false);
    Field nrm = ws_field(c, "fg_nrm", P_F64);
    apply_mpc(c, P_F64, true, bt, nrm, false);
    const double rn2 = dnorm2(c, t2), nb2 = dnorm2(c, nrm);
    double r2 = 0, b2 = 0;
    for (int par = 0; par < 2; par++) {
        Field xp = par ? x : xe, xq = par ? xe : x, bp = par ? bo : be;
        launch_slocal(c, P_F64, SL_A, xq, ax);
        StencilSpec d5;
        d5.out_parity = par;
        d5.self = true;
        d5.s0 = c.d;
        d5.s1 = c.e;
        d5.tau = -0.5;
        launch_stencil(c, P_F64, d5, ax, xp, t2);
        launch_axpby(c, P_F64, 1.0, bp, -1.0, t2, t2);
        r2 += dnorm2(c, t2);
        b2 += dnorm2(c, bp);
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double t3w = wall();
    if (st) {
        st->iters = it;
        st->reliable_updates = 0;
        st->converged = conv ? 1 : 0;
        st->fell_back = 0;
        st->res_normal = nb2 > 0 ? std::sqrt(rn2 / nb2) : 0;
        st->res_schur = bt2 > 0 ? std::sqrt(rs2 / bt2) : 0;
        st->res_full = b2 > 0 ? std::sqrt(r2 / b2) : 0;
        st->seconds = t3w - t0;
        st->t_prep = t1w - t0;
        st->t_solve = t2w - t1w;
        st->t_final = t3w - t2w;
    }
    return status;
    DWF_API_END
}
