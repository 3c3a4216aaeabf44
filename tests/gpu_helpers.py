"""Helpers for the GPU parity tests: contexts from seeded inputs, transfers."""
import numpy as np

import oracle
from oracle import Params
from paper_2203_17119_amd import dwf, synth

TOL = {dwf.DWF_F64: 1e-12, dwf.DWF_F32: 1e-6, dwf.DWF_F16: 2e-3, dwf.DWF_BF16: 1.5e-2}


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
