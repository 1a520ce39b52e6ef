"""The GMRES driver of the Krylov use of the map, on the CPU with dense
operators: it solves a nonsymmetric system to the tolerance (checked with
numpy's solver), restarts correctly, and right preconditioning by the exact
inverse converges in one iteration."""
import numpy as np
import torch

from paper_2406_17656_amd.krylov import gmres


def system(n=60, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    return torch.as_tensor(A), torch.as_tensor(b)


def test_gmres_matches_direct_solve():
    A, b = system()
    x, its, hist = gmres(lambda v: A @ v, lambda v: v, b, tol=1e-10, restart=20, maxiter=500)
    xs = np.linalg.solve(A.numpy(), b.numpy())
    assert np.linalg.norm(x.numpy() - xs) <= 1e-8 * np.linalg.norm(xs)
    assert hist[-1] <= 1e-9 and its > 20          # needed a restart


def test_exact_right_preconditioner_one_step():
    A, b = system(seed=1)
    Ainv = torch.as_tensor(np.linalg.inv(A.numpy()))
    x, its, _ = gmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-10, restart=10, maxiter=50)
    assert its == 1
    assert np.allclose((A @ x).numpy(), b.numpy(), rtol=1e-9, atol=1e-9)
