"""Pins of the oracle's FP64 discrete adjoint (CPU only): gradients of L = sum (phi_T - phi*)^2
with respect to eps and the per-cell initial supersaturation agree with central finite differences
of the oracle's own forward loss; dL/dU0 is the sum of dL/dU_init; the checkpoint stride does not
change the result."""
import dataclasses

import numpy as np
import pytest

import oracle

N, STEPS, SEED = 36, 120, (18.0, 18.0, 5.0)


def problem(n_fold=6, kappa_N=1.0, eps=0.04):
    p = oracle.Params(nx=N, ny=N, eps=eps, n_fold=n_fold, kappa_N=kappa_N)
    rng = np.random.default_rng(11)
    U = 0.5 + 0.02 * rng.standard_normal((N, N))
    target = oracle.final_phi(dataclasses.replace(p, eps=eps + 0.02), SEED, 1.0, 0.55 + 0 * U, STEPS)
    return p, U, target, rng


@pytest.mark.parametrize("n_fold,kappa_N", [(6, 1.0), (4, 2.0)])
def test_adjoint_eps_matches_central_difference(n_fold, kappa_N):
    p, U, target, _ = problem(n_fold, kappa_N)
    L, gU, ge, phiT = oracle.adjoint(p, SEED, 1.0, U, target, STEPS)
    assert abs(L - oracle.loss(p, SEED, 1.0, U, target, STEPS)) < 1e-12 * L
    d = 1e-5
    fd = (oracle.loss(dataclasses.replace(p, eps=p.eps + d), SEED, 1.0, U, target, STEPS)
          - oracle.loss(dataclasses.replace(p, eps=p.eps - d), SEED, 1.0, U, target, STEPS)) / (2 * d)
    assert abs(fd / ge - 1) < 1e-5


def test_adjoint_initial_supersaturation_directional_difference():
    p, U, target, rng = problem()
    L, gU, ge, _ = oracle.adjoint(p, SEED, 1.0, U, target, STEPS)
    for _ in range(2):
        v = rng.standard_normal(U.shape)
        d = 1e-5
        fd = (oracle.loss(p, SEED, 1.0, U + d * v, target, STEPS)
              - oracle.loss(p, SEED, 1.0, U - d * v, target, STEPS)) / (2 * d)
        assert abs(fd / float((gU * v).sum()) - 1) < 1e-7


def test_adjoint_U0_is_sum_over_cells():
    p, U, target, _ = problem()
    L, gU, ge, _ = oracle.adjoint(p, SEED, 1.0, U, target, STEPS)
    d = 1e-4
    fd = (oracle.loss(p, SEED, 1.0, U + d, target, STEPS) - oracle.loss(p, SEED, 1.0, U - d, target, STEPS)) / (2 * d)
    assert abs(fd / gU.sum() - 1) < 1e-5


def test_adjoint_independent_of_checkpoint_stride():
    p, U, target, _ = problem()
    a = oracle.adjoint(p, SEED, 1.0, U, target, STEPS, stride=0)
    b = oracle.adjoint(p, SEED, 1.0, U, target, STEPS, stride=7)
    c = oracle.adjoint(p, SEED, 1.0, U, target, STEPS, stride=1)
    for other in (b, c):
        assert other[0] == a[0] and other[2] == a[2]
        assert np.array_equal(other[1], a[1])


def test_adjoint_rejects_flow():
    p = oracle.Params(nx=8, ny=8, flow=1)
    L, gU, ge, _ = oracle.adjoint(p, (4.0, 4.0, 2.0), 1.0, np.full((8, 8), 0.5), np.zeros((8, 8)), 3)
    assert np.isnan(L)
