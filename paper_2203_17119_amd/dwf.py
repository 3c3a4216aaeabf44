"""Python binding of ``libdwf.so`` (the C ABI declared in ``include/dwf.h``).

Argument marshalling only: every step of every call runs in the library's HIP
kernels.  Field arguments are torch tensors on the GPU (or raw integer device
addresses); canonical fields are complex128 tensors in the layouts the header
documents.  The library is loaded from this package directory and the import
fails loudly when it has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwf.so")

DWF_OK, DWF_EINVAL, DWF_ENOMEM, DWF_EDEVICE, DWF_ENOCONV, DWF_ENOTSUP = 0, -1, -2, -3, -4, -5
DWF_F64, DWF_F32, DWF_F16, DWF_BF16 = 0, 1, 2, 3
DWF_SOLVE_F64, DWF_SOLVE_MIXED_F32, DWF_SOLVE_MIXED_F16, DWF_SOLVE_MIXED_BF16 = 0, 1, 2, 3
DWF_K_DHOP, DWF_K_STENCIL, DWF_K_SLOCAL, DWF_K_BLAS, DWF_K_NET = 0, 1, 2, 3, 4
DWF_NET_FWD_FP32, DWF_NET_FWD_MFMA_BF16 = 0, 1
DWF_OP_CG, DWF_OP_MULTISHIFT, DWF_OP_RATIONAL, DWF_OP_SCHUR_APPLY, DWF_OP_BOUNDARY = 0, 1, 2, 3, 4
DWF_SCHED_STENCIL_BATCHED = 8
DWF_TUNE_NORMAL, DWF_TUNE_BATCHED = 0, 1
KCLASS_NAMES = {DWF_K_DHOP: "dhop", DWF_K_STENCIL: "stencil", DWF_K_SLOCAL: "slocal",
                DWF_K_BLAS: "blas", DWF_K_NET: "net"}


class dwf_params(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("Ls", C.c_int), ("b", C.c_double), ("c", C.c_double),
                ("M5", C.c_double), ("mf", C.c_double), ("dirichlet", C.c_int * 4)]


class dwf_solver_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("mode", C.c_int), ("delta", C.c_double),
                ("x0_is_guess", C.c_int), ("restart", C.c_int), ("normal", C.c_int), ("fallback", C.c_int),
                ("tile_sb", C.c_int), ("tile_run", C.c_int)]


class dwf_solver_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("converged", C.c_int),
                ("fell_back", C.c_int), ("res_normal", C.c_double), ("res_schur", C.c_double),
                ("res_full", C.c_double), ("seconds", C.c_double), ("t_prep", C.c_double),
                ("t_solve", C.c_double), ("t_final", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DWFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dwf status {status}: {msg}")
        self.status = status


class dwf_rational(C.Structure):
    _fields_ = [("n", C.c_int), ("a0", C.c_double), ("alpha", C.POINTER(C.c_double)),
                ("beta", C.POINTER(C.c_double))]


def make_rational(a0, alpha, beta):
    """A dwf_rational r(x) = a0 + sum_k alpha[k] / (x + beta[k]); the returned
    object keeps its coefficient arrays alive."""
    n = len(alpha)
    if len(beta) != n:
        raise ValueError("alpha and beta differ in length")
    al = (C.c_double * n)(*[float(a) for a in alpha])
    be = (C.c_double * n)(*[float(b) for b in beta])
    r = dwf_rational(n, float(a0), al, be)
    r._keep = (al, be)
    return r


class dwf_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_CTX = C.c_void_p
_NET = C.c_void_p

# name -> (argtypes, restype); mirrors include/dwf.h
SIGNATURES = {
    "dwf_abi_version": ([], C.c_int),
    "dwf_last_error": ([], C.c_char_p),
    "dwf_create": ([C.POINTER(dwf_params), _P, _I, _P, C.POINTER(_CTX)], C.c_int32),
    "dwf_destroy": ([_CTX], C.c_int32),
    "dwf_set_gauge": ([_CTX, _P, _I], C.c_int32),
    "dwf_set_stream": ([_CTX, _P], C.c_int32),
    "dwf_field_bytes": ([_CTX, _I, _I, C.POINTER(C.c_size_t)], C.c_int32),
    "dwf_workspace_bytes": ([_CTX, _I, _I, _I, _I, C.POINTER(C.c_size_t)], C.c_int32),
    "dwf_set_workspace": ([_CTX, _P, C.c_size_t], C.c_int32),
    "dwf_workspace_used": ([_CTX, C.POINTER(C.c_size_t)], C.c_int32),
    "dwf_prepare_links": ([_CTX, _I], C.c_int32),
    "dwf_import": ([_CTX, _I, _I, _P, _P], C.c_int32),
    "dwf_export": ([_CTX, _I, _I, _P, _P], C.c_int32),
    "dwf_dhop": ([_CTX, _I, _I, _P, _P], C.c_int32),
    "dwf_dhop_internal": ([_CTX, _I, _I, _I, _P, _P], C.c_int32),
    "dwf_mooee": ([_CTX, _I, _P, _P], C.c_int32),
    "dwf_mooeeinv": ([_CTX, _I, _P, _P], C.c_int32),
    "dwf_schur_apply": ([_CTX, _I, _P, _P], C.c_int32),
    "dwf_schur_apply_internal": ([_CTX, _I, _I, _P, _P], C.c_int32),
    "dwf_schur_apply_internal_noalloc": ([_CTX, _I, _I, _P, _P], C.c_int32),
    "dwf_cg": ([_CTX, _P, _P, C.POINTER(dwf_solver_opts), C.POINTER(dwf_solver_stats)], C.c_int32),
    "dwf_multishift_cg": ([_CTX, _I, C.POINTER(_P), _I, C.POINTER(_D), C.POINTER(_P),
                           C.POINTER(dwf_solver_opts), C.POINTER(dwf_solver_stats)], C.c_int32),
    "dwf_rational_apply": ([_CTX, C.POINTER(dwf_rational), _P, _P, C.POINTER(dwf_solver_opts),
                            C.POINTER(dwf_solver_stats)], C.c_int32),
    "dwf_ddrhmc_action": ([_CTX, _CTX, C.POINTER(dwf_rational), C.POINTER(dwf_rational), _P,
                           C.POINTER(dwf_solver_opts), C.POINTER(_D), C.POINTER(dwf_solver_stats)], C.c_int32),
    "dwf_chebyshev_filter": ([_CTX, _I, _P, _D, _D, _I, C.POINTER(_I), C.POINTER(_P)], C.c_int32),
    "dwf_precond_apply_internal": ([_CTX, _NET, _I, _P, _I, _P], C.c_int32),
    "dwf_mask_links": ([_CTX, _P, _P, _P], C.c_int32),
    "dwf_d5_apply": ([_CTX, _P, _P], C.c_int32),
    "dwf_boundary_project": ([_CTX, _P, _P, _P], C.c_int32),
    "dwf_boundary_apply": ([_CTX, _CTX, _P, _I, _P, _P, C.POINTER(dwf_solver_opts), C.POINTER(dwf_solver_stats)],
                           C.c_int32),
    "dwf_net_create": ([_CTX, _I, C.POINTER(_I), C.POINTER(_NET)], C.c_int32),
    "dwf_net_destroy": ([_NET], C.c_int32),
    "dwf_net_num_weights": ([_NET], C.c_int),
    "dwf_net_set_weights": ([_NET, _P], C.c_int32),
    "dwf_net_get_weights": ([_NET, _P], C.c_int32),
    "dwf_precond_apply": ([_CTX, _NET, _P, _P], C.c_int32),
    "dwf_net_set_forward": ([_NET, _I], C.c_int32),
    "dwf_net_backward": ([_NET, _P, _P, _P, _P], C.c_int32),
    "dwf_net_train_step": ([_NET, _I, C.POINTER(_P), C.POINTER(_P), C.POINTER(dwf_adam), C.POINTER(_D)], C.c_int32),
    "dwf_fgcr": ([_CTX, _NET, _P, _P, C.POINTER(dwf_solver_opts), C.POINTER(dwf_solver_stats)], C.c_int32),
    "dwf_set_site_order": ([_CTX, _I, _I, _I], C.c_int32),
    "dwf_get_site_order": ([_CTX, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)], C.c_int32),
    "dwf_set_tile_schedule": ([_CTX, _I, _I, _I], C.c_int32),
    "dwf_get_tile_schedule": ([_CTX, _I, C.POINTER(_I), C.POINTER(_I)], C.c_int32),
    "dwf_tune": ([_CTX, _I, C.c_char_p, C.POINTER(_D)], C.c_int32),
    "dwf_tune_op": ([_CTX, _I, _I, _I, C.c_char_p, C.POINTER(_D)], C.c_int32),
    "dwf_stream_copy": ([_CTX, _P, _P, C.c_size_t], C.c_int32),
    "dwf_stream_probe": ([_CTX, _I, _I, _I, _P, _P, _P, C.c_size_t], C.c_int32),
    "dwf_kernel_timing": ([_CTX, _I], C.c_int32),
    "dwf_kernel_timing_reset": ([_CTX], C.c_int32),
    "dwf_kernel_timing_mask": ([_CTX, _I], C.c_int32),
    "dwf_kernel_stats": ([_CTX, _I, _I, C.POINTER(C.c_long), C.POINTER(_D), C.POINTER(_D), C.POINTER(_D)], C.c_int32),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises when it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build the HIP library (paper_2203_17119_amd/build.py)")
        # torch ships its own HIP runtime under the same soname as the system
        # one; load it first so that libdwf.so binds to that single runtime and
        # shares devices, streams and allocations with torch
        import torch

        torch.cuda.is_available()
        lib = C.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(status, allow=()):
    if status != DWF_OK and status not in allow:
        raise DWFError(status, load().dwf_last_error().decode())
    return status


def _ptr(t):
    """Device address of a tensor (must be contiguous) or an integer address."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("field tensors must be contiguous")
    return t.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ------------------------------------------------------------- C-ABI mirrors

def dwf_abi_version() -> int:
    return load().dwf_abi_version()


def dwf_last_error() -> str:
    return load().dwf_last_error().decode()


def dwf_create(dims, Ls, b, c, M5, mf, dirichlet, gauge, stream=None):
    """gauge: canonical complex128 tensor [V][4][3][3] on the GPU, or a numpy array (host)."""
    p = dwf_params((C.c_int * 4)(*dims), Ls, b, c, M5, mf, (C.c_int * 4)(*dirichlet))
    ctx = _CTX()
    if isinstance(gauge, np.ndarray):
        g = np.ascontiguousarray(gauge, dtype=np.complex128)
        st = load().dwf_create(C.byref(p), g.ctypes.data, 0, _stream_ptr(stream), C.byref(ctx))
    else:
        st = load().dwf_create(C.byref(p), _ptr(gauge), 1, _stream_ptr(stream), C.byref(ctx))
    _check(st)
    return ctx


def dwf_destroy(ctx):
    _check(load().dwf_destroy(ctx))


def dwf_set_gauge(ctx, gauge):
    if isinstance(gauge, np.ndarray):
        g = np.ascontiguousarray(gauge, dtype=np.complex128)
        _check(load().dwf_set_gauge(ctx, g.ctypes.data, 0))
    else:
        _check(load().dwf_set_gauge(ctx, _ptr(gauge), 1))


def dwf_set_stream(ctx, stream):
    _check(load().dwf_set_stream(ctx, _stream_ptr(stream)))


def dwf_field_bytes(ctx, full, prec) -> int:
    n = C.c_size_t()
    _check(load().dwf_field_bytes(ctx, int(full), int(prec), C.byref(n)))
    return n.value


def dwf_workspace_bytes(ctx, op, mode=DWF_SOLVE_F64, nrhs=1, nshift=1) -> int:
    n = C.c_size_t()
    _check(load().dwf_workspace_bytes(ctx, int(op), int(mode), int(nrhs), int(nshift), C.byref(n)))
    return n.value


def dwf_set_workspace(ctx, ws, nbytes=None):
    """ws: a device tensor (its storage is used; keep it alive while set) or None."""
    if ws is None:
        _check(load().dwf_set_workspace(ctx, None, 0))
    else:
        n = ws.numel() * ws.element_size() if nbytes is None else int(nbytes)
        _check(load().dwf_set_workspace(ctx, _ptr(ws), n))


def dwf_workspace_used(ctx) -> int:
    n = C.c_size_t()
    _check(load().dwf_workspace_used(ctx, C.byref(n)))
    return n.value


def dwf_prepare_links(ctx, prec):
    _check(load().dwf_prepare_links(ctx, int(prec)))


def dwf_import(ctx, full, prec, canon, internal):
    _check(load().dwf_import(ctx, int(full), int(prec), _ptr(canon), _ptr(internal)))


def dwf_export(ctx, full, prec, internal, canon):
    _check(load().dwf_export(ctx, int(full), int(prec), _ptr(internal), _ptr(canon)))


def dwf_dhop(ctx, out_parity, dagger, in_half, out_half):
    _check(load().dwf_dhop(ctx, int(out_parity), int(dagger), _ptr(in_half), _ptr(out_half)))


def dwf_dhop_internal(ctx, prec, out_parity, dagger, inp, out):
    _check(load().dwf_dhop_internal(ctx, int(prec), int(out_parity), int(dagger), _ptr(inp), _ptr(out)))


def dwf_mooee(ctx, dagger, in_half, out_half):
    _check(load().dwf_mooee(ctx, int(dagger), _ptr(in_half), _ptr(out_half)))


def dwf_mooeeinv(ctx, dagger, in_half, out_half):
    _check(load().dwf_mooeeinv(ctx, int(dagger), _ptr(in_half), _ptr(out_half)))


def dwf_schur_apply(ctx, dagger, in_odd, out_odd):
    _check(load().dwf_schur_apply(ctx, int(dagger), _ptr(in_odd), _ptr(out_odd)))


def dwf_schur_apply_internal(ctx, prec, dagger, inp, out):
    _check(load().dwf_schur_apply_internal(ctx, int(prec), int(dagger), _ptr(inp), _ptr(out)))


def dwf_schur_apply_internal_noalloc(ctx, prec, dagger, inp, out):
    _check(load().dwf_schur_apply_internal_noalloc(ctx, int(prec), int(dagger), _ptr(inp), _ptr(out)))


def _opts(tol=1e-8, maxit=0, mode=DWF_SOLVE_F64, delta=0.0, x0_is_guess=False, restart=0, normal=False,
          fallback=True, tile_sb=0, tile_run=1):
    return dwf_solver_opts(tol, maxit, mode, delta, int(x0_is_guess), restart, int(normal), int(fallback),
                           int(tile_sb), int(tile_run))


def dwf_cg(ctx, b_full, x_full, **opts):
    """Full red-black solve D5 x = b.  Returns (status, stats dict); status DWF_ENOCONV is not raised."""
    o = _opts(**opts)
    st = dwf_solver_stats()
    s = _check(load().dwf_cg(ctx, _ptr(b_full), _ptr(x_full), C.byref(o), C.byref(st)), allow=(DWF_ENOCONV,))
    return s, st.asdict()


def dwf_multishift_cg(ctx, b_odd, shifts, x_odd, **opts):
    """b_odd: list of nrhs odd fields; x_odd: list of nrhs*nshift fields (rhs-major)."""
    nrhs, ns = len(b_odd), len(shifts)
    if len(x_odd) != nrhs * ns:
        raise ValueError("need nrhs * nshift solution fields")
    bp = (_P * nrhs)(*[_ptr(t) for t in b_odd])
    xp = (_P * (nrhs * ns))(*[_ptr(t) for t in x_odd])
    sh = (_D * ns)(*[float(s) for s in shifts])
    o = _opts(**opts)
    st = (dwf_solver_stats * (nrhs * ns))()
    s = _check(load().dwf_multishift_cg(ctx, nrhs, bp, ns, sh, xp, C.byref(o), st), allow=(DWF_ENOCONV,))
    return s, [x.asdict() for x in st]


def dwf_rational_apply(ctx, r, in_odd, out_odd, **opts):
    """out = r(A) in, A = Mpc^+ Mpc; r from make_rational.  Returns (status, stats of the worst shift)."""
    o = _opts(**opts)
    st = dwf_solver_stats()
    s = _check(load().dwf_rational_apply(ctx, C.byref(r), _ptr(in_odd), _ptr(out_odd), C.byref(o), C.byref(st)),
               allow=(DWF_ENOCONV,))
    return s, st.asdict()


def dwf_mask_links(ctx, mask, gauge_in, gauge_out):
    """gauge_out = gauge_in with the links between the domains of mask (int8, 1 on Omega) zeroed."""
    _check(load().dwf_mask_links(ctx, _ptr(mask), _ptr(gauge_in), _ptr(gauge_out)))


def dwf_d5_apply(ctx, in_full, out_full):
    """out = D5 in on canonical FP64 full fields."""
    _check(load().dwf_d5_apply(ctx, _ptr(in_full), _ptr(out_full)))


def dwf_boundary_project(ctx, mask, in_full, out_full):
    """out = P in, the projector onto what the boundary hop from Omega sees."""
    _check(load().dwf_boundary_project(ctx, _ptr(mask), _ptr(in_full), _ptr(out_full)))


def dwf_boundary_apply(ctx, ctx_cut, mask, in_full, out_full, inverse=False, **opts):
    """out = R psi or R^-1 psi (inverse).  Returns (status, stats summed over the solves)."""
    o = _opts(**opts)
    st = dwf_solver_stats()
    s = _check(load().dwf_boundary_apply(ctx, ctx_cut, _ptr(mask), int(bool(inverse)), _ptr(in_full),
                                         _ptr(out_full), C.byref(o), C.byref(st)), allow=(DWF_ENOCONV,))
    return s, st.asdict()


def dwf_ddrhmc_action(ctx, ctx_dirichlet, r_quarter, r_minus_half, phi_odd, **opts):
    """S = phi^+ r_q(A_d) r_m(A) r_q(A_d) phi.  Returns (status, S, [stats of r_q, stats of r_m])."""
    o = _opts(**opts)
    st = (dwf_solver_stats * 2)()
    S = C.c_double()
    s = _check(load().dwf_ddrhmc_action(ctx, ctx_dirichlet, C.byref(r_quarter), C.byref(r_minus_half),
                                        _ptr(phi_odd), C.byref(o), C.byref(S), st), allow=(DWF_ENOCONV,))
    return s, S.value, [x.asdict() for x in st]


def dwf_chebyshev_filter(ctx, v_odd, lo, hi, orders, out_odd, prec=DWF_F64):
    """out_odd[i] = T_{orders[i]}(x(A)) v_odd, A = Mpc^+ Mpc, x(A) = (2A - (hi + lo)) / (hi - lo)."""
    n = len(orders)
    if len(out_odd) != n:
        raise ValueError("need one output field per order")
    op = (_P * n)(*[_ptr(t) for t in out_odd])
    oa = (_I * n)(*[int(k) for k in orders])
    _check(load().dwf_chebyshev_filter(ctx, int(prec), _ptr(v_odd), float(lo), float(hi), n, oa, op))


def dwf_net_create(ctx, chans):
    arr = (C.c_int * len(chans))(*chans)
    net = _NET()
    _check(load().dwf_net_create(ctx, len(chans) - 1, arr, C.byref(net)))
    return net


def dwf_net_destroy(net):
    _check(load().dwf_net_destroy(net))


def dwf_net_num_weights(net) -> int:
    return load().dwf_net_num_weights(net)


def dwf_net_set_weights(net, w):
    """w: complex array of dwf_net_num_weights(net) weights, layer blocks [pi][a][b]."""
    a = np.ascontiguousarray(np.asarray(w).ravel(), dtype=np.complex64)
    if a.size != dwf_net_num_weights(net):
        raise ValueError("wrong number of weights")
    _check(load().dwf_net_set_weights(net, a.ctypes.data))


def dwf_net_get_weights(net):
    a = np.empty(dwf_net_num_weights(net), dtype=np.complex64)
    _check(load().dwf_net_get_weights(net, a.ctypes.data))
    return a


def dwf_net_set_forward(net, mode):
    _check(load().dwf_net_set_forward(net, int(mode)))


def dwf_precond_apply(ctx, net, in_odd, out_odd):
    _check(load().dwf_precond_apply(ctx, net, _ptr(in_odd), _ptr(out_odd)))


def dwf_precond_apply_internal(ctx, net, in_prec, inp, out_prec, out):
    """The preconditioner on internal odd fields of the given storage precisions."""
    _check(load().dwf_precond_apply_internal(ctx, net, int(in_prec), _ptr(inp), int(out_prec), _ptr(out)))


def dwf_net_backward(net, in_odd, grad_out_odd, grad_in_odd=None, want_w=True):
    gw = np.empty(dwf_net_num_weights(net), dtype=np.complex64) if want_w else None
    _check(load().dwf_net_backward(net, _ptr(in_odd), _ptr(grad_out_odd), _ptr(grad_in_odd),
                                   gw.ctypes.data if gw is not None else None))
    return gw


def dwf_net_train_step(net, b_odd, x_odd, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, update=True):
    n = len(b_odd)
    bp = (_P * n)(*[_ptr(t) for t in b_odd])
    xp = (_P * n)(*[_ptr(t) for t in x_odd])
    opt = dwf_adam(lr, beta1, beta2, eps)
    loss = C.c_double()
    _check(load().dwf_net_train_step(net, n, bp, xp, C.byref(opt) if update else None, C.byref(loss)))
    return loss.value


def dwf_fgcr(ctx, net, b_full, x_full, **opts):
    o = _opts(**opts)
    st = dwf_solver_stats()
    s = _check(load().dwf_fgcr(ctx, net, _ptr(b_full), _ptr(x_full), C.byref(o), C.byref(st)),
               allow=(DWF_ENOCONV,))
    return s, st.asdict()


def dwf_set_site_order(ctx, cx, cy, cz):
    _check(load().dwf_set_site_order(ctx, int(cx), int(cy), int(cz)))


def dwf_get_site_order(ctx):
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(load().dwf_get_site_order(ctx, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def dwf_set_tile_schedule(ctx, kclass, sites_per_group, xcd_run):
    _check(load().dwf_set_tile_schedule(ctx, int(kclass), int(sites_per_group), int(xcd_run)))


def dwf_get_tile_schedule(ctx, kclass):
    s, r = C.c_int(), C.c_int()
    _check(load().dwf_get_tile_schedule(ctx, int(kclass), C.byref(s), C.byref(r)))
    return s.value, r.value


def dwf_tune(ctx, prec, cache_path=None):
    """Autotune the stencil schedule for prec; returns the chosen schedule's time (ms)."""
    ms = C.c_double()
    _check(load().dwf_tune(ctx, int(prec), cache_path.encode() if cache_path else None, C.byref(ms)))
    return ms.value


def dwf_tune_op(ctx, op, prec, nrhs=1, cache_path=None):
    """Autotune the single-field (DWF_TUNE_NORMAL) or batched (DWF_TUNE_BATCHED,
    nrhs fields) stencil schedule; returns the chosen schedule's time (ms)."""
    ms = C.c_double()
    _check(load().dwf_tune_op(ctx, int(op), int(prec), int(nrhs), cache_path.encode() if cache_path else None,
                              C.byref(ms)))
    return ms.value


def dwf_stream_copy(ctx, src, dst, nbytes):
    _check(load().dwf_stream_copy(ctx, _ptr(src), _ptr(dst), int(nbytes)))


def dwf_stream_probe(ctx, kind, unroll, nontemporal, a, b, dst, nbytes):
    _check(load().dwf_stream_probe(ctx, int(kind), int(unroll), int(nontemporal), _ptr(a), _ptr(b), _ptr(dst),
                                   int(nbytes)))


def dwf_kernel_timing(ctx, enable):
    _check(load().dwf_kernel_timing(ctx, int(enable)))


def dwf_kernel_timing_mask(ctx, mask):
    _check(load().dwf_kernel_timing_mask(ctx, int(mask)))


def dwf_kernel_timing_reset(ctx):
    _check(load().dwf_kernel_timing_reset(ctx))


def dwf_kernel_stats(ctx, kclass, prec=-1):
    n, ms, by, fl = C.c_long(), C.c_double(), C.c_double(), C.c_double()
    _check(load().dwf_kernel_stats(ctx, int(kclass), int(prec), C.byref(n), C.byref(ms), C.byref(by),
                                   C.byref(fl)))
    return {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}


# ------------------------------------------------------------- convenience

class Lattice:
    """Owns a library context for one workload; methods forward to the C ABI."""

    def __init__(self, dims, Ls, b, c, M5, mf, dirichlet=(0, 0, 0, 0), gauge=None, stream=None):
        self.dims, self.Ls = tuple(dims), int(Ls)
        self.b, self.c, self.M5, self.mf = float(b), float(c), float(M5), float(mf)
        self.dirichlet = tuple(dirichlet)
        self.ctx = dwf_create(dims, Ls, b, c, M5, mf, dirichlet, gauge, stream)

    @property
    def V(self):
        return int(np.prod(self.dims))

    def full_shape(self):
        return (self.V, self.Ls, 4, 3)

    def half_shape(self):
        return (self.V // 2, self.Ls, 4, 3)

    def internal(self, prec, full=False):
        """Uninitialised internal field buffer of precision prec (a uint8 tensor)."""
        import torch
        return torch.empty(dwf_field_bytes(self.ctx, full, prec), dtype=torch.uint8, device="cuda")

    def close(self):
        if self.ctx:
            dwf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
