"""ctypes front end of the C oracle (``oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Every function takes and returns numpy complex128 arrays in the canonical
layouts (see ``oracle.c``).  The library is compiled with gcc by ``build()``;
``lib()`` compiles it on first use when it is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
SO = os.path.join(HERE, "liboracle.so")

_lib = None

_d = C.c_double
_i = C.c_int
_l = C.c_long
_p = C.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        tmp = SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(SO)
        sig = {
            "or_gamma": [_i, _p],
            "or_dirichlet": [_p, _p, _p, _p],
            "or_hop": [_p, _i, _p, _p, _p, _i],
            "or_dw": [_p, _i, _d, _p, _p, _p, _i],
            "or_p5": [_l, _i, _d, _p, _p, _i],
            "or_d5": [_p, _i, _d, _d, _d, _d, _p, _p, _p, _i],
            "or_pick": [_p, _i, _p, _i, _p],
            "or_embed": [_p, _i, _p, _i, _p],
            "or_mooee": [_l, _i, _d, _d, _d, _d, _p, _p, _i],
            "or_mooeeinv": [_l, _i, _d, _d, _d, _d, _p, _p, _i],
            "or_meo": [_p, _i, _d, _d, _d, _d, _p, _p, _i, _p, _i],
            "or_mpc": [_p, _i, _d, _d, _d, _d, _p, _p, _p, _i],
            "or_cgne": [_p, _i, _d, _d, _d, _d, _p, _p, _p, _d, _i, _i, _p],
            "or_schur_source": [_p, _i, _d, _d, _d, _d, _p, _p, _p],
            "or_multishift": [_p, _i, _d, _d, _d, _d, _p, _p, _i, _p, _p, _d, _i, _p, _p],
            "or_ptc_layer": [_p, _i, _p, _i, _i, _p, _p, _p],
            "or_ptc_layer_backward": [_p, _i, _p, _i, _i, _p, _p, _p, _p, _p],
            "or_net_apply": [_p, _i, _p, _i, _p, _p, _p, _p],
            "or_fgcr": [_p, _i, _d, _d, _d, _d, _p, _i, _p, _p, _p, _p, _d, _i, _i, _i, _p],
            "or_hop_sites": [_p, _i, _p, _p, _p, _l, _p, _i],
            "or_d5_sites": [_p, _i, _d, _d, _d, _d, _p, _p, _p, _l, _p],
            "or_num_threads": [],
            "or_set_num_threads": [_i],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _i if name in ("or_cgne", "or_multishift", "or_fgcr", "or_num_threads") else None
        _lib = L
    return _lib


def num_threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's following parallel loops."""
    lib().or_set_num_threads(int(n))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dims(L):
    return np.ascontiguousarray(L, dtype=np.int32)


class Params:
    """Moebius domain-wall parameters on a 4D lattice of extents L (all even)."""

    def __init__(self, L, Ls, b, c, M5, mf):
        self.L = tuple(int(x) for x in L)
        self.Ls, self.b, self.c, self.M5, self.mf = int(Ls), float(b), float(c), float(M5), float(mf)
        self._L = _dims(self.L)

    @property
    def V(self):
        return int(np.prod(self.L))

    def full_shape(self):
        return (self.V, self.Ls, 4, 3)

    def half_shape(self):
        return (self.V // 2, self.Ls, 4, 3)

    def args(self):
        return (self.b, self.c, self.M5, self.mf)


def gamma(mu: int) -> np.ndarray:
    """gamma_mu (mu = 0..3 for x,y,z,t) or gamma_5 (mu = 4), 4x4."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().or_gamma(mu, _ptr(out))
    return out


def dirichlet(L, U, mask) -> np.ndarray:
    U = _c128(U)
    out = np.empty_like(U)
    lib().or_dirichlet(_ptr(_dims(L)), _ptr(np.ascontiguousarray(mask, dtype=np.int32)), _ptr(U), _ptr(out))
    return out


def hop(P: Params, U, psi, dagger=False) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_hop(_ptr(P._L), P.Ls, _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def dw(P: Params, U, psi, dagger=False) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_dw(_ptr(P._L), P.Ls, P.M5, _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def p5(P: Params, psi, dagger=False) -> np.ndarray:
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_p5(psi.shape[0], P.Ls, P.mf, _ptr(psi), _ptr(out), int(dagger))
    return out


def d5(P: Params, U, psi, dagger=False) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_d5(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def hop_sites(P: Params, U, psi, sites, dagger=False) -> np.ndarray:
    """(H psi)(n) for the listed lexicographic 4D sites n; shape (len(sites), Ls, 4, 3)."""
    U, psi = _c128(U), _c128(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), P.Ls, 4, 3), dtype=np.complex128)
    lib().or_hop_sites(_ptr(P._L), P.Ls, _ptr(U), _ptr(psi), _ptr(sites), len(sites), _ptr(out), int(dagger))
    return out


def d5_sites(P: Params, U, psi, sites) -> np.ndarray:
    """(D5 psi)(n) for the listed lexicographic 4D sites n; shape (len(sites), Ls, 4, 3)."""
    U, psi = _c128(U), _c128(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), P.Ls, 4, 3), dtype=np.complex128)
    lib().or_d5_sites(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(psi), _ptr(sites), len(sites), _ptr(out))
    return out


def pick(P: Params, full, parity) -> np.ndarray:
    full = _c128(full)
    out = np.empty(P.half_shape(), dtype=np.complex128)
    lib().or_pick(_ptr(P._L), P.Ls, _ptr(full), int(parity), _ptr(out))
    return out


def embed(P: Params, half, parity) -> np.ndarray:
    half = _c128(half)
    out = np.empty(P.full_shape(), dtype=np.complex128)
    lib().or_embed(_ptr(P._L), P.Ls, _ptr(half), int(parity), _ptr(out))
    return out


def mooee(P: Params, psi, dagger=False) -> np.ndarray:
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_mooee(psi.shape[0], P.Ls, *P.args(), _ptr(psi), _ptr(out), int(dagger))
    return out


def mooeeinv(P: Params, psi, dagger=False) -> np.ndarray:
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_mooeeinv(psi.shape[0], P.Ls, *P.args(), _ptr(psi), _ptr(out), int(dagger))
    return out


def meo(P: Params, U, half, p_in, dagger=False) -> np.ndarray:
    """Block of D5 (or D5^+) from parity p_in to parity 1-p_in."""
    U, half = _c128(U), _c128(half)
    out = np.empty(P.half_shape(), dtype=np.complex128)
    lib().or_meo(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(half), int(p_in), _ptr(out), int(dagger))
    return out


def mpc(P: Params, U, odd, dagger=False) -> np.ndarray:
    U, odd = _c128(U), _c128(odd)
    out = np.empty_like(odd)
    lib().or_mpc(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(odd), _ptr(out), int(dagger))
    return out


def schur_source(P: Params, U, b_full) -> np.ndarray:
    U, b_full = _c128(U), _c128(b_full)
    out = np.empty(P.half_shape(), dtype=np.complex128)
    lib().or_schur_source(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(b_full), _ptr(out))
    return out


def cgne(P: Params, U, b_full, tol, maxit=100000, x0=None):
    """Red-black CGNE solve of D5 x = b. Returns (x_full, iters, [res_normal, res_schur, res_full])."""
    U, b_full = _c128(U), _c128(b_full)
    x = np.zeros_like(b_full) if x0 is None else _c128(x0).copy()
    res = np.zeros(3)
    it = lib().or_cgne(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(b_full), _ptr(x), float(tol), int(maxit),
                       int(x0 is not None), _ptr(res))
    return x, it, res


def multishift(P: Params, U, b_odd, shifts, tol, maxit=100000):
    """Multi-shift CG on Mpc^+Mpc + sigma_k.  Returns (x[k], base_iters, iters_k, res_k)."""
    U, b_odd = _c128(U), _c128(b_odd)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    n = len(shifts)
    x = np.zeros((n,) + b_odd.shape, dtype=np.complex128)
    iters = np.zeros(n, dtype=np.int32)
    res = np.zeros(n)
    it = lib().or_multishift(_ptr(P._L), P.Ls, *P.args(), _ptr(U), _ptr(b_odd), n, _ptr(shifts), _ptr(x),
                             float(tol), int(maxit), _ptr(iters), _ptr(res))
    return x, it, iters, res


def chebyshev(P: Params, U, v_odd, lo, hi, orders):
    """Chebyshev filter of A = Mpc^+ Mpc on [lo, hi] (the recursively generated
    filter functions for multigrid subspace set-up, Sec. 2.4): with
    x(A) = (2A - (hi + lo)) / (hi - lo), the three-term recurrence
    T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1} applied to v.
    Returns [T_k(x(A)) v for k in orders] (orders ascending)."""
    v = _c128(v_odd)
    a, sh = 2.0 / (hi - lo), -(hi + lo) / (hi - lo)

    def xa(w):
        return a * mpc(P, U, mpc(P, U, w), True) + sh * w

    out, want = [], list(orders)
    wm, w0 = None, v.copy()
    for k in range(max(want) + 1):
        if k == 1:
            wm, w0 = w0, xa(w0)
        elif k >= 2:
            wm, w0 = w0, 2.0 * xa(w0) - wm
        while want and want[0] == k:
            out.append(w0.copy())
            want.pop(0)
    return out


NPATH = 11


def ptc_layer(L, Ls, U, W, phi):
    """One parallel-transport convolution layer. W: (11, Cout, Cin); phi: (V, Ls, Cin, 3)."""
    U, W, phi = _c128(U), _c128(W), _c128(phi)
    npath, cout, cin = W.shape
    out = np.empty(phi.shape[:2] + (cout, 3), dtype=np.complex128)
    lib().or_ptc_layer(_ptr(_dims(L)), int(Ls), _ptr(U), cin, cout, _ptr(W), _ptr(phi), _ptr(out))
    return out


def ptc_layer_backward(L, Ls, U, W, phi, gout, want_in=True, want_w=True):
    """Real-pair gradients (dL/dRe + i dL/dIm) of one layer: returns (g_in, g_W)."""
    U, W, phi, gout = _c128(U), _c128(W), _c128(phi), _c128(gout)
    npath, cout, cin = W.shape
    gin = np.empty_like(phi) if want_in else None
    gW = np.zeros_like(W) if want_w else None
    lib().or_ptc_layer_backward(_ptr(_dims(L)), int(Ls), _ptr(U), cin, cout, _ptr(W), _ptr(phi), _ptr(gout),
                                _ptr(gin), _ptr(gW))
    return gin, gW


def net_apply(P: Params, U, weights, odd):
    """Network preconditioner on an odd half field. weights: list of (11, Cout, Cin) arrays."""
    U, odd = _c128(U), _c128(odd)
    chans = np.array([weights[0].shape[2]] + [w.shape[1] for w in weights], dtype=np.int32)
    W = np.concatenate([_c128(w).ravel() for w in weights])
    out = np.empty_like(odd)
    lib().or_net_apply(_ptr(P._L), P.Ls, _ptr(U), len(weights), _ptr(chans), _ptr(W), _ptr(odd), _ptr(out))
    return out


def fgcr(P: Params, U, b_odd, tol, maxit=10000, m=16, weights=None, normal=False):
    """Flexible GCR(m) on Mpc x = b (or Mpc^+ Mpc x = b when ``normal``), optionally
    right-preconditioned by the network."""
    U, b_odd = _c128(U), _c128(b_odd)
    x = np.zeros_like(b_odd)
    res = np.zeros(1)
    if weights:
        chans = np.array([weights[0].shape[2]] + [w.shape[1] for w in weights], dtype=np.int32)
        W = np.concatenate([_c128(w).ravel() for w in weights])
        nl = len(weights)
    else:
        chans = np.zeros(1, dtype=np.int32)
        W = np.zeros(1, dtype=np.complex128)
        nl = 0
    it = lib().or_fgcr(_ptr(P._L), P.Ls, *P.args(), _ptr(U), nl, _ptr(chans), _ptr(W), _ptr(b_odd), _ptr(x),
                       float(tol), int(maxit), int(m), int(normal), _ptr(res))
    return x, it, res[0]


def adam_step(w, g, m, v, step, lr, beta1, beta2, eps):
    """One Adam update (Kingma & Ba, "Adam: a method for stochastic
    optimization", Algorithm 1) on real FP64 arrays, elementwise:
        m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
        m^ = m / (1 - beta1^t),   v^ = v / (1 - beta2^t),
        w <- w - lr m^ / (sqrt(v^) + eps)
    with t = step (1 for the first update).  Complex weights are updated as
    their (re, im) pairs with the real-pair gradient dL/dRe + i dL/dIm.
    Returns (w, m, v) as new arrays."""
    w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------- DD-RHMC
#
# The one-flavour boundary action of Sec. 2.3.1, eq. (ddrhmc):
#     S = phi^+ (D_d^+ D_d)^{1/4} (D^+ D)^{-1/2} (D_d^+ D_d)^{1/4} phi
# with D the operator of the whole lattice and D_d the Dirichlet one of the
# same field.  On the odd sites of the red-black system the normal operators
# are A = Mpc^+ Mpc and A_d = Mpc_d^+ Mpc_d: det D5 = det Mee det Mpc and Mee
# is site- and field-independent, so the determinant ratio the action samples
# is the same.  The oracle evaluates the matrix functions exactly from the
# eigendecomposition of the dense Hermitian matrices (small lattices only).


def dense_normal(P: Params, U) -> np.ndarray:
    """Dense A = Mpc^+ Mpc on the odd half field, built column by column."""
    n = int(np.prod(P.half_shape()))
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = mpc(P, U, e.reshape(P.half_shape())).ravel()
        e[j] = 0.0
    return M.conj().T @ M


def herm_power(A, p):
    """A^p of a Hermitian positive definite matrix from its eigendecomposition."""
    lam, V = np.linalg.eigh(A)
    if lam[0] <= 0:
        raise ValueError("matrix not positive definite")
    return (V * lam ** p) @ V.conj().T


def rational_dense(A, a0, alpha, beta):
    """r(A) = a0 + sum_k alpha_k (A + beta_k)^-1 for a dense matrix A."""
    n = A.shape[0]
    out = a0 * np.eye(n, dtype=np.complex128)
    for al, be in zip(alpha, beta):
        out += al * np.linalg.inv(A + be * np.eye(n))
    return out


def ddrhmc_action(P: Params, U_full, U_dirichlet, phi_odd, quarter=None, minus_half=None):
    """S = phi^+ f(A_d) g(A) f(A_d) phi with f(x) = x^{1/4}, g(x) = x^{-1/2}
    (exact, by eigendecomposition), or with the rational functions given as
    (a0, alpha, beta) tuples in their place.  Returns the real action."""
    A = dense_normal(P, U_full)
    Ad = dense_normal(P, U_dirichlet)
    f = herm_power(Ad, 0.25) if quarter is None else rational_dense(Ad, *quarter)
    g = herm_power(A, -0.5) if minus_half is None else rational_dense(A, *minus_half)
    v = np.asarray(phi_odd, dtype=np.complex128).ravel()
    psi = f @ v
    return float(np.real(np.vdot(psi, g @ psi)))


# ------------------------------------------------------------ domain boundary
# Sec. 2.1: the lattice splits into a domain Omega (mask 1) and its complement
# Omega-bar (mask 0).  Ordered by domain, D = [[D_Omega, D_d], [D_dbar,
# D_Omegabar]], with D_d and D_dbar the hops across the domain boundary.  The
# cut operator D_cut = diag(D_Omega, D_Omegabar) is D on the gauge field whose
# links between the domains are zero, so D_d + D_dbar = D - D_cut.
#
# The projector P_dbar keeps the components of a field on Omega that D_dbar
# acts on (D_dbar P_dbar = D_dbar).  With D5 = Mooee - (1/2) H A, a site x of
# Omega feeds Omega-bar only through the hop, which sees (1 + gamma_mu) A psi(x)
# when x + mu is in Omega-bar and (1 - gamma_mu) A psi(x) when x - mu is.  The
# spin-space mask Pi of the boundary is therefore (1 +- gamma_mu)/2 at a site
# with one such neighbour, 1 at a site with two or more (the ranges of two
# different projectors of this kind span the four spins), 0 elsewhere, and
# P_dbar = A^-1 Pi A (A = b + c P5; for Shamir, c = 0, it is Pi itself).


def coords(L, n):
    x = []
    for mu in range(4):
        x.append(n % L[mu])
        n //= L[mu]
    return x


def lexi(L, x):
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))


def mask_cut(L, U, mask):
    """The gauge field with every link U_mu(x) whose ends lie in different domains set to zero."""
    U = np.array(U, dtype=np.complex128, copy=True).reshape(-1, 4, 3, 3)
    mask = np.asarray(mask).ravel()
    for n in range(U.shape[0]):
        x = coords(L, n)
        for mu in range(4):
            y = list(x)
            y[mu] = (y[mu] + 1) % L[mu]
            if mask[n] != mask[lexi(L, y)]:
                U[n, mu] = 0.0
    return U


def boundary_spin_mask(L, mask):
    """Pi per site, shape (V, 4, 4)."""
    mask = np.asarray(mask).ravel()
    V = len(mask)
    one = np.eye(4, dtype=np.complex128)
    Pi = np.zeros((V, 4, 4), dtype=np.complex128)
    for n in range(V):
        if mask[n] != 1:
            continue
        x = coords(L, n)
        links = []
        for mu in range(4):
            for sgn in (1, -1):
                y = list(x)
                y[mu] = (y[mu] + sgn) % L[mu]
                if mask[lexi(L, y)] == 0:
                    links.append((mu, sgn))
        if len(links) == 1:
            mu, sgn = links[0]
            Pi[n] = 0.5 * (one + sgn * gamma(mu))
        elif len(links) > 1:
            Pi[n] = one
    return Pi


def a_site_matrix(P: Params, inverse=False) -> np.ndarray:
    """A = b + c P5 (or its inverse) on the Ls x 4 x 3 components of one 4D site."""
    m = 12 * P.Ls
    E = np.eye(m, dtype=np.complex128).reshape(m, P.Ls, 4, 3)
    A = (P.b * E + P.c * p5(P, E)).reshape(m, m).T  # column j = A e_j
    return np.linalg.inv(A) if inverse else A


def boundary_projector(P: Params, mask, psi) -> np.ndarray:
    """P_dbar psi = A^-1 Pi A psi for a full field psi."""
    V, m = P.V, 12 * P.Ls
    A, Ai = a_site_matrix(P), a_site_matrix(P, inverse=True)
    v = (np.asarray(psi, dtype=np.complex128).reshape(V, m) @ A.T).reshape(V, P.Ls, 4, 3)
    v = np.einsum("nab,nsbc->nsac", boundary_spin_mask(P.L, mask), v)
    return (v.reshape(V, m) @ Ai.T).reshape(P.full_shape())


def dense_d5(P: Params, U) -> np.ndarray:
    """Dense D5 on the full field, built column by column (small lattices only)."""
    n = int(np.prod(P.full_shape()))
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = d5(P, U, e.reshape(P.full_shape())).ravel()
        e[j] = 0.0
    return M


def dense_boundary_projector(P: Params, mask) -> np.ndarray:
    n = int(np.prod(P.full_shape()))
    E = np.eye(n, dtype=np.complex128)
    return np.stack([boundary_projector(P, mask, E[:, j]).ravel() for j in range(n)], axis=1)


def restrict(P: Params, mask, psi) -> np.ndarray:
    """psi on the sites of Omega, zero on Omega-bar."""
    keep = (np.asarray(mask).ravel() == 1).astype(np.float64)
    return np.asarray(psi, dtype=np.complex128).reshape(P.full_shape()) * keep[:, None, None, None]


def boundary_r(P: Params, U, U_cut, mask, psi, inverse=False):
    """R psi = P psi - P D_Omega^-1 D_d D_Omegabar^-1 D_dbar psi, or
    R^-1 psi = P psi - P D^-1 D_dbar psi (Sec. 2.1), by dense solves, for the
    part of psi on Omega (these operators act on fields of Omega).  D_cut^-1
    applied to a field on one domain is that domain's inverse, and D - D_cut
    applied to it is the hop into the other domain."""
    shp = P.full_shape()
    D, Dc = dense_d5(P, U), dense_d5(P, U_cut)
    off = D - Dc
    v = restrict(P, mask, psi).ravel()
    if inverse:
        w = np.linalg.solve(D, off @ v)
    else:
        w = np.linalg.solve(Dc, off @ np.linalg.solve(Dc, off @ v))
    return boundary_projector(P, mask, v.reshape(shp)) - boundary_projector(P, mask, w.reshape(shp))
