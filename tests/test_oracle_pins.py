"""The FP64 oracle against what the mathematics and the paper fix (CPU only)."""
import numpy as np
import pytest
import torch

import pins
from paper_2302_09224_amd import inputs


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(check, oracle_lib):
    ok, detail = check(oracle_lib)
    assert ok, detail


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8), (4, 8, 6, 4)])
@pytest.mark.parametrize("kind", ["haar", "near_unit"])
def test_antihermitian_shapes(dims, kind, oracle_lib):
    # 4^4 included on purpose: there x+3mu and x-mu are the same site
    ok, detail = pins.check_antihermitian(oracle_lib, dims=dims, kind=kind)
    assert ok, detail


def test_haar_generator():
    gen = torch.Generator().manual_seed(3)
    u = inputs.haar_su3(20000, gen)
    eye = torch.eye(3, dtype=torch.complex128)
    assert (u.conj().transpose(-1, -2) @ u - eye).abs().max() < 1e-13
    assert (torch.linalg.det(u) - 1).abs().max() < 1e-13
    # Haar moments: E|U_ij|^2 = 1/3, E tr U = 0, E|tr U|^2 = 1
    assert abs((u.abs() ** 2).mean().item() - 1 / 3) < 3e-3
    tr = torch.diagonal(u, dim1=-2, dim2=-1).sum(-1)
    assert tr.mean().abs().item() < 0.03
    assert abs((tr.abs() ** 2).mean().item() - 1.0) < 0.04


def test_near_unit_generator():
    gen = torch.Generator().manual_seed(4)
    u = inputs.near_unit_su3(5000, gen)
    eye = torch.eye(3, dtype=torch.complex128)
    assert (u.conj().transpose(-1, -2) @ u - eye).abs().max() < 1e-13
    assert (torch.linalg.det(u) - 1).abs().max() < 1e-13
    # exp(i eps H): eigenphases are eps * eigenvalues of a traceless H
    ph = torch.angle(torch.linalg.eigvals(u))
    assert ph.sum(-1).abs().max() < 1e-10
    dist = (u - eye).abs().max(-1).values.max(-1).values
    assert 0.05 < dist.mean().item() < 0.6


def test_link_structure():
    dims = (4, 4, 4, 6)
    fat, lng = inputs.make_links(dims, "haar", seed=9, fold_phases=False)
    eye = torch.eye(3, dtype=torch.complex128)
    l24 = -24.0 * lng
    assert (l24.conj().transpose(-1, -2) @ l24 - eye).abs().max() < 1e-13   # L = -U1U2U3/24
    assert (torch.linalg.det(l24) - 1).abs().max() < 1e-12
    ff = fat.conj().transpose(-1, -2) @ fat
    assert (ff - eye).abs().max() > 0.1                                       # F is not unitary
    assert torch.linalg.matrix_norm(fat, ord=2).max() <= 1.0 + 1e-12          # |0.6U+0.4U'| <= 1
    f2, l2 = inputs.make_links(dims, "haar", seed=9)
    eta_f, eta_l = inputs.eta_phases(dims)
    assert torch.equal(f2, fat * eta_f.reshape(4, -1, 1, 1))
    assert torch.equal(l2, lng * eta_l.reshape(4, -1, 1, 1))


def test_seeds_reproducible():
    a = inputs.make_links((4, 4, 4, 4), "near_unit", seed=5)
    b = inputs.make_links((4, 4, 4, 4), "near_unit", seed=5)
    c = inputs.make_links((4, 4, 4, 4), "near_unit", seed=6)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert not torch.equal(a[0], c[0])
