// C ABI of the library: context lifetime, gauge preparation, workspaces,
// kernel timing and the operator entry points.  Solvers live in solvers.cpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dwf_internal.h"

using namespace dwf;

namespace dwf {

static thread_local std::string g_err;

void set_error(const std::string &m) { g_err = m; }

[[noreturn]] void fail(dwf_status code, const std::string &m) { throw Error{code, m}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(DWF_ENOMEM, std::string(what) + ": out of device memory");
        fail(DWF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

size_t elem_bytes(int prec)
{
    switch (prec) {
    case P_F64: return 16;
    case P_F32: return 8;
    default: return 4;
    }
}

size_t field_bytes(const Context &c, long n5, int prec)
{
    (void)c;
    size_t b = (size_t)12 * n5 * elem_bytes(prec);
    if (prec == P_F16) b += (size_t)n5 * sizeof(float);
    return b;
}

Field make_field(const Context &c, void *data, int prec)
{
    Field f;
    f.data = data;
    f.n = c.n5h;
    f.norm = (prec == P_F16) ? (float *)((char *)data + (size_t)12 * c.n5h * elem_bytes(prec)) : nullptr;
    return f;
}

// device memory for a workspace buffer: carved from the caller's workspace
// when one is set, else allocated (and then owned) by the library
static void *ws_alloc(Context &c, size_t bytes, bool &owned)
{
    if (c.uws) {
        const size_t off = (c.uws_used + 255) & ~(size_t)255;
        if (off + bytes > c.uws_bytes)
            fail(DWF_ENOMEM, "caller workspace too small: " + std::to_string(off + bytes) + " bytes needed, " +
                                 std::to_string(c.uws_bytes) + " given (dwf_workspace_bytes)");
        c.uws_used = off + bytes;
        owned = false;
        return c.uws + off;
    }
    void *p = nullptr;
    HIPCHECK(hipMalloc(&p, bytes));
    owned = true;
    return p;
}

static Context::Buf &ws_get(Context &c, const std::string &key, size_t bytes, int prec)
{
    auto it = c.ws.find(key);
    if (it == c.ws.end()) {
        Context::Buf b;
        b.bytes = bytes;
        b.data = ws_alloc(c, bytes, b.owned);
        HIPCHECK(hipMemsetAsync(b.data, 0, b.bytes, c.stream));
        b.prec = prec;
        it = c.ws.emplace(key, b).first;
    }
    return it->second;
}

Field ws_field(Context &c, const std::string &name, int prec)
{
    const std::string key = name + "#" + std::to_string(prec);
    return make_field(c, ws_get(c, key, field_bytes(c, c.n5h, prec), prec).data, prec);
}

void *ws_raw(Context &c, const std::string &name, size_t bytes)
{
    Context::Buf &b = ws_get(c, name + "#raw", bytes, -1);
    if (b.bytes < bytes) fail(DWF_EINVAL, "workspace buffer " + name + " reused with a larger size");
    return b.data;
}

size_t ws_plan_bytes(const Context &c, const std::vector<WsKey> &plan)
{
    size_t total = 0;
    std::vector<std::string> seen;
    for (const WsKey &k : plan) {
        const std::string key = k.prec < 0 ? k.name + "#raw"
                                : k.nbatch <= 1 ? k.name + "#" + std::to_string(k.prec)
                                                : k.name + "#" + std::to_string(k.prec) + "x" + std::to_string(k.nbatch);
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
        seen.push_back(key);
        size_t b = k.prec < 0 ? k.raw
                   : k.nbatch <= 1 ? field_bytes(c, c.n5h, k.prec)
                                   : (size_t)batch_stride(c, k.prec) * k.nbatch;
        total += (b + 255) & ~(size_t)255;
    }
    return total;
}

const void *slmat(const Context &c, int op, bool f64)
{
    const size_t off = (size_t)op * 2 * c.Ls * c.Ls;
    return f64 ? (const void *)(c.slmat64 + off) : (const void *)(c.slmat32 + off);
}

Timer::Timer(Context &c_, int k, double by, double fl, int pr) : c(c_), kclass(k), prec(pr), bytes(by), flops(fl)
{
    if (!(c.timing >> k & 1)) return;
    if (c.event_pool.empty()) {
        hipEvent_t e;
        HIPCHECK(hipEventCreate(&e));
        c.event_pool.push_back(e);
    }
    a = c.event_pool.back();
    c.event_pool.pop_back();
    HIPCHECK(hipEventRecord(a, c.stream));
}

Timer::~Timer()
{
    if (!a) return;
    if (c.event_pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c.event_pool.push_back(e);
    }
    hipEvent_t b = c.event_pool.back();
    c.event_pool.pop_back();
    if (hipEventRecord(b, c.stream) != hipSuccess) return;
    c.pending.push_back(TimedLaunch{kclass, prec, a, b, bytes, flops});
}

static void drain_timing(Context &c)
{
    if (c.pending.empty()) return;
    HIPCHECK(hipStreamSynchronize(c.stream));
    for (auto &t : c.pending) {
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, t.a, t.b));
        for (int k = 0; k < 2; k++) {
            if (k == 1 && (t.prec < 0 || t.prec > 3)) break;
            KStats &s = k == 0 ? c.stats[t.kclass] : c.stats_prec[t.kclass][t.prec];
            s.launches++;
            s.ms += ms;
            s.bytes += t.bytes;
            s.flops += t.flops;
        }
        c.event_pool.push_back(t.a);
        c.event_pool.push_back(t.b);
    }
    c.pending.clear();
}

void read_scalars(Context &c, int first, int count)
{
    HIPCHECK(hipMemcpyAsync(c.hscal + first, c.dscal + first, count * sizeof(double), hipMemcpyDeviceToHost,
                            c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
}

// ----------------------------------------------------- s-local matrices

// Upper (P+) and lower (P-) blocks of the fifth-dimension operators.  P5 moves
// the P+ spins from s-1 and the P- spins from s+1, with -mf at the walls.
static void build_slocal(Context &c)
{
    const int n = c.Ls;
    const double mf = c.p.mf, b = c.p.b, cc = c.p.c, d = c.d, e = c.e;
    auto idx = [n](int r, int col) { return (size_t)r * n + col; };
    std::vector<double> Sup(n * n, 0.0), Slo(n * n, 0.0), I(n * n, 0.0);
    for (int s = 0; s < n; s++) {
        I[idx(s, s)] = 1.0;
        if (s >= 1) Sup[idx(s, s - 1)] += 1.0;
        else Sup[idx(0, n - 1)] += -mf;
        if (s + 1 < n) Slo[idx(s, s + 1)] += 1.0;
        else Slo[idx(n - 1, 0)] += -mf;
    }
    auto lin = [&](double a0, double a1, const std::vector<double> &S) {
        std::vector<double> m(n * n);
        for (size_t k = 0; k < m.size(); k++) m[k] = a0 * I[k] + a1 * S[k];
        return m;
    };
    auto mul = [&](const std::vector<double> &A, const std::vector<double> &B) {
        std::vector<double> m(n * n, 0.0);
        for (int r = 0; r < n; r++)
            for (int k = 0; k < n; k++)
                for (int col = 0; col < n; col++) m[idx(r, col)] += A[idx(r, k)] * B[idx(k, col)];
        return m;
    };
    auto tr = [&](const std::vector<double> &A) {
        std::vector<double> m(n * n);
        for (int r = 0; r < n; r++)
            for (int col = 0; col < n; col++) m[idx(r, col)] = A[idx(col, r)];
        return m;
    };
    // closed-form inverse of d + e S_up: S_up^n = -mf, so
    // (d + e S)^-1 = sum_k (-e/d)^k S^k / (d (1 + mf (-e/d)^n))
    std::vector<double> Minv(n * n);
    const double al = -e / d;
    const double norm = d * (1.0 + mf * std::pow(al, n));
    for (int s = 0; s < n; s++)
        for (int t = 0; t < n; t++)
            Minv[idx(s, t)] = (s >= t) ? std::pow(al, s - t) / norm : -mf * std::pow(al, s - t + n) / norm;
    // (b + c S_up)^-1 in the same closed form (zero when b = 0: the boundary
    // operators then refuse the parameters)
    std::vector<double> Ainv(n * n, 0.0);
    if (b != 0.0) {
        const double ga = -cc / b;
        const double an = b * (1.0 + mf * std::pow(ga, n));
        for (int s = 0; s < n; s++)
            for (int t = 0; t < n; t++)
                Ainv[idx(s, t)] = (s >= t) ? std::pow(ga, s - t) / an : -mf * std::pow(ga, s - t + n) / an;
    }
    std::vector<std::vector<double>> blocks(2 * SL_NOP);
    auto setop = [&](int op, const std::vector<double> &up, const std::vector<double> &lo) {
        blocks[2 * op] = up;
        blocks[2 * op + 1] = lo;
    };
    setop(SL_A, lin(b, cc, Sup), lin(b, cc, Slo));
    setop(SL_ADAG, lin(b, cc, Slo), lin(b, cc, Sup));
    setop(SL_MOOEE, lin(d, e, Sup), lin(d, e, Slo));
    setop(SL_MOOEEDAG, lin(d, e, Slo), lin(d, e, Sup));
    setop(SL_MINV, Minv, tr(Minv));
    setop(SL_MINVDAG, tr(Minv), Minv);
    setop(SL_E1, mul(blocks[2 * SL_A], blocks[2 * SL_MINV]), mul(blocks[2 * SL_A + 1], blocks[2 * SL_MINV + 1]));
    setop(SL_E2, mul(blocks[2 * SL_MINVDAG], blocks[2 * SL_ADAG]),
          mul(blocks[2 * SL_MINVDAG + 1], blocks[2 * SL_ADAG + 1]));
    setop(SL_AINV, Ainv, tr(Ainv));
    // twisted-circulant operators (polynomials in the shift, per chirality):
    // T[t][s] = f_{t-s} (t >= s), -mf f_{t-s+n} (t < s), the other block T^T
    auto twisted = [&](const std::vector<double> &T, const std::vector<double> &O, double *f) {
        double scale = 0;
        for (double v : T) scale = std::max(scale, std::fabs(v));
        if (scale == 0) return false;
        for (int k = 0; k < n; k++) f[k] = T[idx(k, 0)];
        for (int t = 0; t < n; t++)
            for (int col = 0; col < n; col++) {
                const double want = t >= col ? f[t - col] : -mf * f[t - col + n];
                if (std::fabs(T[idx(t, col)] - want) > 1e-12 * scale) return false;
                if (std::fabs(O[idx(col, t)] - T[idx(t, col)]) > 1e-12 * scale) return false;
            }
        return true;
    };
    // first column of (beta + gamma S)(delta + eps S)^-1, S = S_up
    auto rational_column = [&](double be, double ga, double de, double ep, double *f) {
        const double r = -ep / de;
        const double nrm = de * (1.0 + mf * std::pow(r, n));
        for (int k = 0; k < n; k++) {
            const double y = std::pow(r, k) / nrm;                         // (delta + eps S)^-1, column 0
            const double y1 = k >= 1 ? std::pow(r, k - 1) / nrm : 0.0;     // shifted by one
            f[k] = be * y + ga * y1;
        }
    };
    const double cand[4][4] = {{b, cc, d, e}, {1.0, 0.0, d, e}, {b, cc, 1.0, 0.0}, {d, e, 1.0, 0.0}};
    for (int op = 0; op < SL_NOP; op++) {
        c.toep_ok[op] = false;
        c.toep_rev[op] = 0;
        c.toep_rat[op] = false;
        if (n > 16) continue;
        if (twisted(blocks[2 * op], blocks[2 * op + 1], c.toep_f[op])) {
            c.toep_ok[op] = true;
        } else if (twisted(blocks[2 * op + 1], blocks[2 * op], c.toep_f[op])) {
            c.toep_ok[op] = true;
            c.toep_rev[op] = 1;
        }
        if (!c.toep_ok[op]) continue;
        double fs = 0;
        for (int k = 0; k < n; k++) fs = std::max(fs, std::fabs(c.toep_f[op][k]));
        for (const auto &q : cand) {
            if (q[2] == 0.0 || std::fabs(q[3] / q[2]) > 0.5) continue;
            double fr[16];
            rational_column(q[0], q[1], q[2], q[3], fr);
            bool same = true;
            for (int k = 0; k < n; k++) same = same && std::fabs(fr[k] - c.toep_f[op][k]) <= 1e-12 * fs;
            if (same) {
                c.toep_rat[op] = true;
                for (int k = 0; k < 4; k++) c.toep_rc[op][k] = q[k];
                break;
            }
        }
    }
    std::vector<double> h64;
    std::vector<float> h32;
    for (auto &bl : blocks)
        for (double v : bl) {
            h64.push_back(v);
            h32.push_back((float)v);
        }
    if (!c.slmat64) HIPCHECK(hipMalloc(&c.slmat64, h64.size() * sizeof(double)));
    if (!c.slmat32) HIPCHECK(hipMalloc(&c.slmat32, h32.size() * sizeof(float)));
    HIPCHECK(hipMemcpy(c.slmat64, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(c.slmat32, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice));
}

static void upload_gauge(Context &c, const double *gauge, int on_device)
{
    const size_t bytes = (size_t)c.V4 * 4 * 9 * 16;
    if (!c.gauge_canon) HIPCHECK(hipMalloc(&c.gauge_canon, bytes));
    HIPCHECK(hipMemcpyAsync(c.gauge_canon, gauge, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c.stream));
    for (int prec = 0; prec < 4; prec++)
        if (prec == P_F64 || c.links[prec][0]) prepare_links(c, prec);
    HIPCHECK(hipStreamSynchronize(c.stream));
}

void ensure_links(Context &c, int prec)
{
    if (!c.links[prec][0]) prepare_links(c, prec);
}

// default stencil schedule: each XCD sweeps whole columns of the site order
void default_schedule(Context &c)
{
    const int sb = default_sb(c);
    const long col = column_sites(c);
    c.cfg_stencil.sb = 0;
    c.cfg_stencil.run = (col < c.vh && col % sb == 0) ? (int)std::min<long>(col / sb, 1 << 20) : 1;
    c.cfg_stencil_batch = c.cfg_stencil;
}

// ---------------------------------------------------------------- Mpc

long batch_stride(const Context &c, int prec) { return (long)((field_bytes(c, c.n5h, prec) + 255) / 256 * 256); }

Field ws_batch(Context &c, const std::string &name, int prec, int nbatch)
{
    if (nbatch <= 1) return ws_field(c, name, prec);
    const std::string key = name + "#" + std::to_string(prec) + "x" + std::to_string(nbatch);
    return make_field(c, ws_get(c, key, (size_t)batch_stride(c, prec) * nbatch, prec).data, prec);
}

int apply_mpc(Context &c, int prec, bool dagger, Field in, Field out, bool reduce, bool in_is_A_applied, Field pa,
              int nbatch, long bstride, int alpha_slot, Field ws_ta, Field ws_y)
{
    if (alpha_slot >= 0 && (!dagger || nbatch > 1)) fail(DWF_EINVAL, "fused residual update needs Mpc^+, one field");
    ensure_links(c, prec);
    const int nb = std::max(1, nbatch);
    Field y = ws_y.data ? ws_y : ws_batch(c, "mpc_y", prec, nb);
    if (nb > 1 && bstride != batch_stride(c, prec)) fail(DWF_EINVAL, "batched fields must use the batch stride");
    auto batched = [&](StencilSpec &s) {
        s.nbatch = nb;
        s.bstride = bstride;
    };
    if (!dagger) {
        Field ta = pa;
        if (!in_is_A_applied) {
            ta = ws_ta.data ? ws_ta : ws_batch(c, "mpc_ta", prec, nb);
            launch_slocal(c, prec, SL_A, in, ta, nb, bstride);
        }
        StencilSpec s1;
        s1.out_parity = 0;
        s1.epi = EPI_DENSE;
        s1.epi_op = SL_E1;
        batched(s1);
        launch_stencil(c, prec, s1, ta, Field{}, y);
        StencilSpec s2;
        s2.out_parity = 1;
        s2.self = true;
        s2.s0 = c.d;
        s2.s1 = c.e;
        s2.tau = -0.25;
        s2.reduce = reduce;
        batched(s2);
        return launch_stencil(c, prec, s2, y, in, out);
    }
    StencilSpec s1;
    s1.out_parity = 0;
    s1.dagger = true;
    s1.epi = EPI_DENSE;
    s1.epi_op = SL_E2;
    batched(s1);
    launch_stencil(c, prec, s1, in, Field{}, y);
    StencilSpec s2;
    s2.out_parity = 1;
    s2.dagger = true;
    s2.epi = EPI_SHIFT;
    s2.e0 = c.p.b;
    s2.e1 = c.p.c;
    s2.edag = true;
    s2.self = true;
    s2.s0 = c.d;
    s2.s1 = c.e;
    s2.sdag = true;
    s2.tau = -0.25;
    s2.reduce = reduce || alpha_slot >= 0;
    s2.cg_update = alpha_slot >= 0;
    s2.alpha_slot = alpha_slot;
    batched(s2);
    return launch_stencil(c, prec, s2, y, in, out);
}

int launch_stencil_f64(Context &, const StencilSpec &, Field, Field, Field);
int launch_stencil_f32(Context &, const StencilSpec &, Field, Field, Field);
int launch_stencil_f16(Context &, const StencilSpec &, Field, Field, Field);
int launch_stencil_bf16(Context &, const StencilSpec &, Field, Field, Field);
void launch_slocal_f64(Context &, int, Field, Field, int, long);
void launch_slocal_f32(Context &, int, Field, Field, int, long);
void launch_slocal_f16(Context &, int, Field, Field, int, long);
void launch_slocal_bf16(Context &, int, Field, Field, int, long);

int launch_stencil(Context &c, int prec, const StencilSpec &sp, Field in, Field self, Field out)
{
    ensure_links(c, prec);
    switch (prec) {
    case P_F64: return launch_stencil_f64(c, sp, in, self, out);
    case P_F32: return launch_stencil_f32(c, sp, in, self, out);
    case P_F16: return launch_stencil_f16(c, sp, in, self, out);
    default: return launch_stencil_bf16(c, sp, in, self, out);
    }
}

void launch_slocal(Context &c, int prec, int op, Field in, Field out, int nbatch, long bstride)
{
    // the operators of the form e0 + e1 P5 need only the fifth-dimension neighbours
    if (op == SL_A || op == SL_ADAG) return launch_slocal_shift(c, prec, c.p.b, c.p.c, op == SL_ADAG, in, out, nbatch, bstride);
    if (op == SL_MOOEE || op == SL_MOOEEDAG)
        return launch_slocal_shift(c, prec, c.d, c.e, op == SL_MOOEEDAG, in, out, nbatch, bstride);
    switch (prec) {
    case P_F64: launch_slocal_f64(c, op, in, out, nbatch, bstride); break;
    case P_F32: launch_slocal_f32(c, op, in, out, nbatch, bstride); break;
    case P_F16: launch_slocal_f16(c, op, in, out, nbatch, bstride); break;
    default: launch_slocal_bf16(c, op, in, out, nbatch, bstride); break;
    }
}

}  // namespace dwf

// ================================================================ C ABI

static void check_prec(int prec)
{
    if (prec < 0 || prec > 3) fail(DWF_EINVAL, "unknown precision");
}

static dwf::Context &C_(dwf_ctx ctx)
{
    if (!ctx) fail(DWF_EINVAL, "null context");
    return *ctx;
}

static void require(const void *p, const char *what)
{
    if (!p) fail(DWF_EINVAL, std::string("null pointer: ") + what);
}

extern "C" {

int dwf_abi_version(void) { return 1; }

const char *dwf_last_error(void) { return dwf::g_err.c_str(); }

dwf_status dwf_create(const dwf_params *p, const double *gauge, int gauge_on_device, void *stream, dwf_ctx *out)
{
    DWF_API_BEGIN
    require(p, "params");
    require(gauge, "gauge");
    require(out, "out");
    *out = nullptr;
    for (int mu = 0; mu < 4; mu++)
        if (p->dims[mu] < 2 || (p->dims[mu] & 1)) fail(DWF_EINVAL, "every lattice extent must be even and >= 2");
    if (p->Ls < 1) fail(DWF_EINVAL, "Ls must be >= 1");
    if (p->Ls > 64) fail(DWF_ENOTSUP, "Ls > 64 is not supported");
    if (!std::isfinite(p->b) || !std::isfinite(p->c) || !std::isfinite(p->M5) || !std::isfinite(p->mf))
        fail(DWF_EINVAL, "non-finite operator parameter");
    const double dd = p->b * (4.0 - p->M5) + 1.0;
    if (dd == 0.0) fail(DWF_EINVAL, "b(4-M5)+1 = 0: Mooee is singular");
    long V4 = (long)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
    if (V4 * p->Ls / 2 > (1L << 30)) fail(DWF_ENOTSUP, "lattice too large for 32-bit neighbour indices");
    auto *c = new dwf_context();
    try {
        c->p = *p;
        for (int mu = 0; mu < 4; mu++) c->L[mu] = p->dims[mu];
        c->Ls = p->Ls;
        c->V4 = V4;
        c->vh = V4 / 2;
        c->n5h = c->vh * c->Ls;
        c->d = dd;
        c->e = p->c * (4.0 - p->M5) - 1.0;
        c->stream = (hipStream_t)stream;
        HIPCHECK(hipGetDevice(&c->device));
        scratch_init(c->device);
        {
            int lds = 0;
            HIPCHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
            c->lds_max = std::min<size_t>(65536, (size_t)lds);
        }
        HIPCHECK(hipMalloc(&c->nbr, (size_t)2 * 8 * c->vh * sizeof(int)));
        HIPCHECK(hipMalloc(&c->nbr_sm, (size_t)2 * 8 * c->vh * sizeof(int)));
        build_order(*c, 0, 0, 0);
        build_neighbours(*c);
        default_schedule(*c);
        build_slocal(*c);
        c->partials_len = 2 * (c->n5h / 64 + c->vh + 1024);
        HIPCHECK(hipMalloc(&c->partials, c->partials_len * sizeof(double)));
        HIPCHECK(hipMalloc(&c->dscal, HS_MIRROR * sizeof(double)));
        HIPCHECK(hipMemset(c->dscal, 0, HS_MIRROR * sizeof(double)));
        HIPCHECK(hipHostMalloc(&c->hscal, HS_MIRROR * sizeof(double), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc(&c->hring, 2 * sizeof(double), hipHostMallocCoherent));
        HIPCHECK(hipHostGetDevicePointer((void **)&c->dring, c->hring, 0));
        for (auto &e : c->cg_ev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        upload_gauge(*c, gauge, gauge_on_device);
    } catch (...) {
        dwf_destroy(c);
        throw;
    }
    *out = c;
    DWF_API_END
}

dwf_status dwf_destroy(dwf_ctx ctx)
{
    if (!ctx) return DWF_OK;
    dwf::Context &c = *ctx;
    (void)hipStreamSynchronize(c.stream);
    for (auto &t : c.pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c.event_pool) (void)hipEventDestroy(e);
    for (auto e : c.cg_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &kv : c.ws)
        if (kv.second.owned) (void)hipFree(kv.second.data);
    for (int pr = 0; pr < 4; pr++)
        for (int p = 0; p < 2; p++)
            if (c.links[pr][p]) (void)hipFree(c.links[pr][p]);
    for (int p = 0; p < 2; p++)
        if (c.links_net[p]) (void)hipFree(c.links_net[p]);
    if (c.nbr) (void)hipFree(c.nbr);
    if (c.nbr_sm) (void)hipFree(c.nbr_sm);
    if (c.perm_inv) (void)hipFree(c.perm_inv);
    if (c.slmat64) (void)hipFree(c.slmat64);
    if (c.slmat32) (void)hipFree(c.slmat32);
    if (c.gauge_canon) (void)hipFree(c.gauge_canon);
    if (c.partials) (void)hipFree(c.partials);
    if (c.dscal) (void)hipFree(c.dscal);
    if (c.hscal) (void)hipHostFree(c.hscal);
    if (c.hring) (void)hipHostFree(c.hring);
    delete ctx;
    return DWF_OK;
}

dwf_status dwf_set_workspace(dwf_ctx ctx, void *ws, size_t bytes)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (ws && ((uintptr_t)ws % 256)) fail(DWF_EINVAL, "workspace must be 256-byte aligned");
    HIPCHECK(hipStreamSynchronize(c.stream));
    // buffers carved from the previous caller workspace are forgotten; the
    // library's own allocations stay
    for (auto it = c.ws.begin(); it != c.ws.end();) {
        if (!it->second.owned) it = c.ws.erase(it);
        else ++it;
    }
    c.uws = ws ? (char *)ws : nullptr;
    c.uws_bytes = ws ? bytes : 0;
    c.uws_used = 0;
    DWF_API_END
}

dwf_status dwf_workspace_used(dwf_ctx ctx, size_t *bytes)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    require(bytes, "bytes");
    *bytes = c.uws_used;
    DWF_API_END
}

dwf_status dwf_prepare_links(dwf_ctx ctx, int prec)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    check_prec(prec);
    ensure_links(c, prec);
    HIPCHECK(hipStreamSynchronize(c.stream));
    DWF_API_END
}

dwf_status dwf_set_gauge(dwf_ctx ctx, const double *gauge, int on_device)
{
    DWF_API_BEGIN
    require(gauge, "gauge");
    upload_gauge(C_(ctx), gauge, on_device);
    DWF_API_END
}

dwf_status dwf_set_stream(dwf_ctx ctx, void *stream)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    drain_timing(c);
    HIPCHECK(hipStreamSynchronize(c.stream));
    c.stream = (hipStream_t)stream;
    DWF_API_END
}

dwf_status dwf_field_bytes(dwf_ctx ctx, int full, int prec, size_t *bytes)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    check_prec(prec);
    require(bytes, "bytes");
    *bytes = field_bytes(c, c.n5h, prec) * (full ? 2 : 1);
    DWF_API_END
}

static void import_any(dwf::Context &c, int full, int prec, const double *canon, void *internal)
{
    if (full) {
        const size_t hb = field_bytes(c, c.n5h, prec);
        launch_import(c, prec, canon, make_field(c, internal, prec), 1, 0);
        launch_import(c, prec, canon, make_field(c, (char *)internal + hb, prec), 1, 1);
    } else {
        launch_import(c, prec, canon, make_field(c, internal, prec), 0, 0);
    }
}

dwf_status dwf_import(dwf_ctx ctx, int full, int prec, const double *canon, void *internal)
{
    DWF_API_BEGIN
    check_prec(prec);
    require(canon, "canon");
    require(internal, "internal");
    import_any(C_(ctx), full, prec, canon, internal);
    DWF_API_END
}

dwf_status dwf_export(dwf_ctx ctx, int full, int prec, const void *internal, double *canon)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    check_prec(prec);
    require(canon, "canon");
    require(internal, "internal");
    if (full) {
        const size_t hb = field_bytes(c, c.n5h, prec);
        launch_export(c, prec, make_field(c, (void *)internal, prec), canon, 1, 0);
        launch_export(c, prec, make_field(c, (char *)internal + hb, prec), canon, 1, 1);
    } else {
        launch_export(c, prec, make_field(c, (void *)internal, prec), canon, 0, 0);
    }
    DWF_API_END
}

dwf_status dwf_dhop(dwf_ctx ctx, int out_parity, int dagger, const double *in_half, double *out_half)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    require(in_half, "in");
    require(out_half, "out");
    if (out_parity != 0 && out_parity != 1) fail(DWF_EINVAL, "parity must be 0 or 1");
    Field a = ws_field(c, "io_a", P_F64), b = ws_field(c, "io_b", P_F64);
    launch_import(c, P_F64, in_half, a, 0, 0);
    StencilSpec sp;
    sp.out_parity = out_parity;
    sp.dagger = dagger != 0;
    sp.kclass = DWF_K_DHOP;
    launch_stencil(c, P_F64, sp, a, Field{}, b);
    launch_export(c, P_F64, b, out_half, 0, 0);
    DWF_API_END
}

dwf_status dwf_dhop_internal(dwf_ctx ctx, int prec, int out_parity, int dagger, const void *in, void *out)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    check_prec(prec);
    require(in, "in");
    require(out, "out");
    if (in == out) fail(DWF_EINVAL, "in and out must differ");
    if (out_parity != 0 && out_parity != 1) fail(DWF_EINVAL, "parity must be 0 or 1");
    StencilSpec sp;
    sp.out_parity = out_parity;
    sp.dagger = dagger != 0;
    sp.kclass = DWF_K_DHOP;
    launch_stencil(c, prec, sp, make_field(c, (void *)in, prec), Field{}, make_field(c, out, prec));
    DWF_API_END
}

static dwf_status slocal_api(dwf_ctx ctx, int op, const double *in_half, double *out_half)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    require(in_half, "in");
    require(out_half, "out");
    Field a = ws_field(c, "io_a", P_F64);
    launch_import(c, P_F64, in_half, a, 0, 0);
    launch_slocal(c, P_F64, op, a, a);
    launch_export(c, P_F64, a, out_half, 0, 0);
    DWF_API_END
}

dwf_status dwf_mooee(dwf_ctx ctx, int dagger, const double *in_half, double *out_half)
{
    return slocal_api(ctx, dagger ? SL_MOOEEDAG : SL_MOOEE, in_half, out_half);
}

dwf_status dwf_mooeeinv(dwf_ctx ctx, int dagger, const double *in_half, double *out_half)
{
    return slocal_api(ctx, dagger ? SL_MINVDAG : SL_MINV, in_half, out_half);
}

dwf_status dwf_schur_apply(dwf_ctx ctx, int dagger, const double *in_odd, double *out_odd)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    require(in_odd, "in");
    require(out_odd, "out");
    Field a = ws_field(c, "io_a", P_F64), b = ws_field(c, "io_b", P_F64);
    launch_import(c, P_F64, in_odd, a, 0, 0);
    apply_mpc(c, P_F64, dagger != 0, a, b, false);
    launch_export(c, P_F64, b, out_odd, 0, 0);
    DWF_API_END
}

dwf_status dwf_schur_apply_internal(dwf_ctx ctx, int prec, int dagger, const void *in, void *out)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    check_prec(prec);
    require(in, "in");
    require(out, "out");
    if (in == out) fail(DWF_EINVAL, "in and out must differ");
    apply_mpc(c, prec, dagger != 0, make_field(c, (void *)in, prec), make_field(c, out, prec), false);
    DWF_API_END
}

static LaunchCfg &cfg_of(dwf::Context &c, int kclass)
{
    switch (kclass) {
    case DWF_K_DHOP:
    case DWF_K_STENCIL: return c.cfg_stencil;
    case DWF_SCHED_STENCIL_BATCHED: return c.cfg_stencil_batch;
    case DWF_K_SLOCAL: return c.cfg_slocal;
    default: fail(DWF_EINVAL, "tile schedules exist for DWF_K_STENCIL, DWF_SCHED_STENCIL_BATCHED and DWF_K_SLOCAL");
    }
}

dwf_status dwf_set_tile_schedule(dwf_ctx ctx, int kclass, int sites_per_group, int xcd_run)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (sites_per_group < 0 || (long)sites_per_group * c.Ls > 256)
        fail(DWF_EINVAL, "sites_per_group * Ls must be <= 256");
    if (xcd_run < 1 || xcd_run > (1 << 20)) fail(DWF_EINVAL, "xcd_run must be in [1, 2^20]");
    LaunchCfg &g = cfg_of(c, kclass);
    g.sb = sites_per_group;
    g.run = xcd_run;
    DWF_API_END
}

dwf_status dwf_get_tile_schedule(dwf_ctx ctx, int kclass, int *sites_per_group, int *xcd_run)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    LaunchCfg &g = cfg_of(c, kclass);
    if (sites_per_group) *sites_per_group = g.sb > 0 ? g.sb : default_sb(c);
    if (xcd_run) *xcd_run = g.run;
    DWF_API_END
}

dwf_status dwf_set_site_order(dwf_ctx ctx, int cx, int cy, int cz)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    const bool dflt = cx == 0 && cy == 0 && cz == 0;
    if (!dflt) {
        if (cx < 2 || (cx & 1) || cy < 1 || cz < 1) fail(DWF_EINVAL, "column extents: cx even >= 2, cy, cz >= 1");
        if (c.L[0] % cx || c.L[1] % cy || c.L[2] % cz) fail(DWF_EINVAL, "column extents must divide Lx, Ly, Lz");
    }
    HIPCHECK(hipStreamSynchronize(c.stream));
    build_order(c, dflt ? 0 : cx / 2, cy, cz);
    build_neighbours(c);
    for (int prec = 0; prec < 4; prec++)
        if (c.links[prec][0]) prepare_links(c, prec);
    default_schedule(c);
    HIPCHECK(hipStreamSynchronize(c.stream));
    DWF_API_END
}

dwf_status dwf_get_site_order(dwf_ctx ctx, int *cx, int *cy, int *cz)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (cx) *cx = 2 * c.order[0];
    if (cy) *cy = c.order[1];
    if (cz) *cz = c.order[2];
    DWF_API_END
}

dwf_status dwf_stream_copy(dwf_ctx ctx, const void *src, void *dst, size_t bytes)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    require(src, "src");
    require(dst, "dst");
    if (bytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        fail(DWF_EINVAL, "stream copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    if (bytes) launch_stream_copy(c, src, dst, bytes);
    DWF_API_END
}

dwf_status dwf_stream_probe(dwf_ctx ctx, int kind, int unroll, int nontemporal, const void *a, const void *b,
                            void *dst, size_t bytes)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (kind < 0 || kind > 2) fail(DWF_EINVAL, "probe kind must be 0 (copy), 1 (read) or 2 (two reads, one write)");
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) fail(DWF_EINVAL, "unroll must be 1, 2, 4 or 8");
    require(a, "a");
    require(dst, "dst");
    if (kind == 2) require(b, "b");
    if (bytes % 16 || ((uintptr_t)a % 16) || ((uintptr_t)dst % 16) || (b && (uintptr_t)b % 16))
        fail(DWF_EINVAL, "probes need 16-byte aligned pointers and a multiple of 16 bytes");
    if (bytes) launch_stream_probe(c, kind, unroll, nontemporal != 0, a, b, dst, bytes);
    DWF_API_END
}

dwf_status dwf_kernel_timing(dwf_ctx ctx, int enable)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    drain_timing(c);
    c.timing = enable ? (1 << DWF_K_NCLASS) - 1 : 0;
    DWF_API_END
}

dwf_status dwf_kernel_timing_mask(dwf_ctx ctx, int mask)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (mask < 0 || mask >= (1 << DWF_K_NCLASS)) fail(DWF_EINVAL, "unknown kernel class in mask");
    drain_timing(c);
    c.timing = mask;
    DWF_API_END
}

dwf_status dwf_kernel_timing_reset(dwf_ctx ctx)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    drain_timing(c);
    for (auto &s : c.stats) s = KStats{};
    for (auto &r : c.stats_prec)
        for (auto &s : r) s = KStats{};
    DWF_API_END
}

dwf_status dwf_kernel_stats(dwf_ctx ctx, int kclass, int prec, long *launches, double *ms, double *bytes,
                            double *flops)
{
    DWF_API_BEGIN
    dwf::Context &c = C_(ctx);
    if (kclass < 0 || kclass >= DWF_K_NCLASS) fail(DWF_EINVAL, "unknown kernel class");
    if (prec < -1 || prec > 3) fail(DWF_EINVAL, "unknown precision");
    drain_timing(c);
    const KStats &s = prec < 0 ? c.stats[kclass] : c.stats_prec[kclass][prec];
    if (launches) *launches = s.launches;
    if (ms) *ms = s.ms;
    if (bytes) *bytes = s.bytes;
    if (flops) *flops = s.flops;
    DWF_API_END
}

}  // extern "C"
