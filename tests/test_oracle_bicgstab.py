"""Pins of the oracle's BiCGStab(l) for the whole-lattice operator M = 2m + D:
the dense solve, l = 1 against the textbook BiCGStab recurrence (van der Vorst
1992, written out here independently), the minimal-residual step's
orthogonality, and agreement between l = 1, 2, 4."""
import numpy as np
import pytest

import oracle
from paper_2302_09224_amd import inputs

DIMS = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def system():
    fat, lng = inputs.make_links(DIMS, "haar", seed=inputs.GAUGE_SEED + 70)
    V = oracle.volume(DIMS)
    b = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 70).numpy()
    return fat.numpy(), lng.numpy(), b


def dense_M(fat, lng, mass):
    V = oracle.volume(DIMS)
    n = 3 * V
    A = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros((V, 3), dtype=np.complex128)
    for k in range(n):
        e.flat[k] = 1.0
        A[:, k] = oracle.full_op(fat, lng, e, DIMS, mass).ravel()
        e.flat[k] = 0.0
    return A


def test_full_op_is_2m_plus_antihermitian(system):
    fat, lng, _ = system
    A = dense_M(fat, lng, 0.1)
    D = A - 0.2 * np.eye(A.shape[0])
    assert np.abs(D + D.conj().T).max() < 1e-14


@pytest.mark.parametrize("l", [1, 2, 4])
def test_bicgstab_l_matches_dense_solve(system, l):
    fat, lng, b = system
    mass = 0.1
    xd = np.linalg.solve(dense_M(fat, lng, mass), b.ravel())
    x, k, res, st = oracle.bicgstab_l(fat, lng, b, DIMS, mass, l=l, tol=1e-12)
    assert st == 0 and res <= 1e-12 * (1 + 1e-6)
    assert np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd) < 1e-10


def test_l1_is_textbook_bicgstab(system):
    """BiCGStab(1) and BiCGStab produce the same residuals in exact arithmetic
    (a well-conditioned mass, so that rounding does not amplify over the steps)"""
    fat, lng, b = system
    mass = 2.0
    M = lambda v: oracle.full_op(fat, lng, v, DIMS, mass)
    # textbook BiCGStab
    x = np.zeros_like(b)
    r = b - M(x)
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    ref = []
    for _ in range(8):
        rho_new = np.vdot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = M(p)
        alpha = rho_new / np.vdot(rh, v)
        s = r - alpha * v
        t = M(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        ref.append(np.linalg.norm(r))
    got = []
    oracle.bicgstab_l(fat, lng, b, DIMS, mass, l=1, tol=0.0, maxiter=16,
                      on_mr=lambda r0, rh_: got.append(np.linalg.norm(r0)))
    assert len(got) == 8 and ref[-1] < 1e-3 * ref[0]
    assert np.allclose(got, ref, rtol=1e-9, atol=0)


def test_minimal_residual_step_orthogonality(system):
    fat, lng, b = system
    worst = []

    def hook(r0, rhat):
        for j, a in enumerate(rhat):
            worst.append(abs(np.vdot(a, r0)) / (np.linalg.norm(a) * np.linalg.norm(r0)))
            for c in rhat[:j]:
                worst.append(abs(np.vdot(c, a)) / (np.linalg.norm(a) * np.linalg.norm(c)))
    oracle.bicgstab_l(fat, lng, b, DIMS, 0.05, l=4, tol=1e-10, on_mr=hook)
    assert len(worst) > 0 and max(worst) < 1e-10


def test_l_agree_on_near_unit_6x4(system):
    dims = (6, 4, 4, 6)
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 71)
    b = inputs.gaussian_spinor(oracle.volume(dims), inputs.SOURCE_SEED + 71).numpy()
    xs = []
    for l in (1, 2, 4):
        x, k, res, st = oracle.bicgstab_l(fat.numpy(), lng.numpy(), b, dims, 0.02, l=l, tol=1e-12)
        assert st == 0 and res <= 1e-12 * (1 + 1e-6), (l, res)
        xs.append(x)
    for x in xs[1:]:
        assert np.linalg.norm(x - xs[0]) / np.linalg.norm(xs[0]) < 1e-9
