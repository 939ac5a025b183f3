"""Pins of the unrolled-RTCUR-F oracle (oracle/unrolled.py), the reference
for the library's differentiable pass:

* with the hard threshold (tau = 0) and the geometric schedule
  zeta_k = gamma^k zeta_0 it is Algorithm 1 itself: L^K on the blocks equals
  the NumPy oracle's RTCUR-F after K iterations (whose L-update takes U_i^+
  from LAPACK's SVD rather than from the Gram's eigendecomposition);
* the gate is the closed form D sigmoid((|D|/zeta - 1)/tau) and tends to the
  strict hard threshold away from |D| = zeta;
* its autograd gradient (thresholds and X) agrees with float64 central
  differences of the same function.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import rtcur
from oracle.unrolled import gate, unrolled


def _inst():
    return synth.tucker_plus_sparse((16, 14, 12), (2, 2, 2), alpha=0.15, seed=21)


def test_hard_threshold_geometric_schedule_is_rtcur_f():
    inst = _inst()
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    K, gamma = 6, 0.7
    zeta0 = float(np.max(np.abs(inst.X)))
    ref = rtcur(inst.X, inst.ranks, I, None, zeta0, gamma, 0.0, K, 0, "F")
    zetas = torch.tensor([zeta0 * gamma ** (k + 1) for k in range(K)], dtype=torch.float64)
    # the oracle multiplies repeatedly; the same values
    z = zeta0
    for k in range(K):
        z *= gamma
        zetas[k] = z
    LB = unrolled(torch.from_numpy(inst.X), inst.ranks, I, zetas, 0.0)
    for b, (L, R) in enumerate(zip(LB, ref.LB)):
        err = np.linalg.norm(L.numpy() - R) / np.linalg.norm(R)
        assert err <= 1e-10, (b, err)


def test_gate_closed_form_and_limit():
    D = torch.tensor([-3.0, -1.0, -0.5, 0.0, 0.25, 1.0, 2.0, 5.0], dtype=torch.float64)
    zeta = 1.0
    for tau in (0.5, 0.1):
        want = D * (1.0 / (1.0 + torch.exp(-((D.abs() / zeta - 1.0) / tau))))
        assert torch.allclose(gate(D, zeta, tau), want, rtol=0, atol=1e-15)
    hard = gate(D, zeta, 0.0)
    assert torch.equal(hard, torch.where(D.abs() > zeta, D, torch.zeros_like(D)))
    # |D| = zeta is not kept (strict), and a small tau reproduces the hard
    # threshold away from the boundary
    assert hard[1] == 0.0 and hard[5] == 0.0
    soft = gate(D, zeta, 1e-3)
    away = (D.abs() - zeta).abs() > 0.1
    assert torch.allclose(soft[away], hard[away], atol=1e-12)


def test_autograd_matches_central_differences():
    inst = synth.tucker_plus_sparse((9, 8, 7), (2, 2, 2), alpha=0.15, seed=5)
    I, _ = synth.sample_sizes(inst.dims, inst.ranks, 3.0)
    K, tau = 4, 0.2
    zeta0 = float(np.max(np.abs(inst.X)))
    z0 = torch.tensor([zeta0 * 0.7 ** (k + 1) for k in range(K)], dtype=torch.float64)
    rng = np.random.default_rng(3)
    X0 = torch.from_numpy(inst.X.copy())
    LB0 = unrolled(X0, inst.ranks, I, z0, tau)
    W = [torch.from_numpy(rng.standard_normal(b.shape)) for b in LB0]

    def loss(X, z):
        return sum((w * L).sum() for w, L in zip(W, unrolled(X, inst.ranks, I, z, tau)))

    X = X0.clone().requires_grad_(True)
    z = z0.clone().requires_grad_(True)
    loss(X, z).backward()
    h = 1e-6
    for k in range(K):
        zp, zm = z0.clone(), z0.clone()
        zp[k] += h
        zm[k] -= h
        fd = (loss(X0, zp) - loss(X0, zm)).item() / (2 * h)
        assert math.isclose(fd, z.grad[k].item(), rel_tol=1e-5, abs_tol=1e-7), (k, fd, z.grad[k])
    # a few entries of X (sampled ones carry the gradient)
    flat = X.grad.reshape(-1)
    picks = list(np.argsort(-np.abs(flat.numpy()))[:4]) + [0]
    for e in picks:
        Xp, Xm = X0.clone().reshape(-1), X0.clone().reshape(-1)
        Xp[e] += h
        Xm[e] -= h
        fd = (loss(Xp.reshape(X0.shape), z0) - loss(Xm.reshape(X0.shape), z0)).item() / (2 * h)
        assert math.isclose(fd, flat[e].item(), rel_tol=1e-5, abs_tol=1e-7), (e, fd, flat[e])
