"""Helpers shared by the GPU parity tests: one seeded problem, built on both
the HIP path (through the C-ABI) and the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O
from paper_1303_1377_amd import fields as F


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """max |a - b| / max |b| over all entries."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()


COMMON = ("levels", "n_tv", "agg", "sap", "mr_steps", "nu", "n_inv", "coarse_tol", "coarse_restart", "coarse_maxit",
          "coarse_fixed", "mid_tol", "mid_restart", "mid_maxit", "mid_fixed", "outer_restart", "outer_maxit",
          "id_setup")


class Pair:
    """The same D on the GPU solver and on the oracle."""

    def __init__(self, dims, eps=0.3, seed=0, ape=0, m0=-0.4, csw=1.0, clover_T=None):
        import paper_1303_1377_amd as G

        self.dims = tuple(dims)
        self.vol = int(np.prod(dims))
        self.U = F.make_gauge(dims, eps, seed, ape_steps=ape)
        self.m0, self.csw = m0, csw
        self.o = O.Oracle(dims, self.U, m0, csw, clover_T=clover_T)
        self.g = G.Solver(dims, self.U, m0, csw, clover=clover_T)

    def configure(self, precision=64, **kw):
        import paper_1303_1377_amd as G

        okw = {k: v for k, v in kw.items() if k in COMMON}
        self.o.configure(**okw)
        self.g.configure(G.default_params(precision=precision, **okw))

    def vectors(self, level, n, seed):
        vol, nd = self.o.level_size(level)
        return F.random_vectors(vol, nd, n, seed)
