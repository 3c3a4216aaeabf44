"""Helpers for the GPU parity tests: contexts from seeded inputs, transfers."""
import numpy as np

import oracle
from oracle import Params
from paper_2203_17119_amd import dwf, synth

TOL = {dwf.DWF_F64: 1e-12, dwf.DWF_F32: 1e-6, dwf.DWF_F16: 2e-3, dwf.DWF_BF16: 1.5e-2}
# Bound on the error of any single 5D site, relative to that site's own norm.
# The global norm above averages over 1e4-1e6 sites; a wrong workgroup tail or
# Dirichlet face would spoil a few sites by O(1) and hide in the average.  A
# site's output sums eight neighbour terms, each rounded at the input's
# precision (FP16: 2^-11 of the neighbour's largest component, so several
# times that relative to a small component), plus the output's own rounding.
# Measured worst sites over every test lattice: FP64 4.7e-16, FP32 2.0e-7,
# FP16 5.9e-4, BF16 5.1e-3; the bounds are the global ones.
SITE_TOL = dict(TOL)


def torch():
    import torch as T
    return T


def to_gpu(a):
    T = torch()
    return T.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    torch().cuda.synchronize()
    return t.cpu().numpy()


class Case:
    """A lattice, its Moebius parameters, a seeded gauge field and a GPU context."""

    def __init__(self, dims, Ls, mf=0.01, dirichlet=(0, 0, 0, 0), eps=0.5, seed=1, b=1.5, c=0.5, M5=1.8):
        self.dims, self.Ls = tuple(dims), Ls
        self.P = Params(dims, Ls, b, c, M5, mf)
        self.U = synth.gauge_field(dims, eps, seed)
        self.dirichlet = tuple(dirichlet)
        self.Ud = oracle.dirichlet(dims, self.U, dirichlet)  # the oracle's Dirichlet block field
        self.lat = dwf.Lattice(dims, Ls, b, c, M5, mf, dirichlet, gauge=self.U)
        self.ctx = self.lat.ctx
        self.seed = seed

    def half(self, seed):
        return synth.gaussian_fermion(self.dims, self.Ls, seed, nsites=self.P.V // 2)

    def full(self, seed):
        return synth.gaussian_fermion(self.dims, self.Ls, seed)

    def oracle_dhop(self, half_in, out_parity, dagger):
        f = oracle.embed(self.P, half_in, 1 - out_parity)
        return oracle.pick(self.P, oracle.hop(self.P, self.Ud, f, dagger), out_parity)

    def close(self):
        self.lat.close()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def site_relerr(a, b):
    """Largest relative error of one 5D site (12 spin-colour components),
    for fields shaped [..., Ls, 4, 3] or already [n5, 12]."""
    a = np.asarray(a).reshape(-1, 12)
    b = np.asarray(b).reshape(-1, 12)
    nb = np.linalg.norm(b, axis=1)
    keep = nb > 1e-6 * nb.max()  # sites whose exact output vanishes carry no relative error
    return float((np.linalg.norm(a - b, axis=1)[keep] / nb[keep]).max())
