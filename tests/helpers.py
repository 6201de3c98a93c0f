"""Shared helpers for the GPU parity tests: seeded inputs rounded to the
precision the GPU receives, so that the oracle and the HIP path start from
identical values."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_1203_4587_amd import synthetic as S


def c64(a: np.ndarray) -> np.ndarray:
    """Round to complex64 and back to complex128 (the GPU's input precision)."""
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


class Case:
    """A synthetic problem with its measured data, all rounded to complex64."""

    def __init__(self, problem):
        self.p = problem
        self.coil = c64(problem.coil)
        self.mask = problem.mask.copy()
        self.x_true = c64(problem.x_true)
        self.y = c64(O.forward(self.x_true, self.coil, self.mask) + problem.noise)

    def device(self):
        import torch
        from paper_1203_4587_amd.api import to_device
        return (to_device(self.coil), to_device(self.mask, dtype=torch.uint8), to_device(self.y))


def make_case(nv, nh, nt, nc, accel=4, ncenter=4, prior="tv", family="cardiac", seed=0, **kw):
    return Case(S.make_problem(nv, nh, nt, nc, accel, ncenter, prior, family, seed, **kw))
