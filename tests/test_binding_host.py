"""Host-side logic of the Python binding (no GPU): the autograd function's check that the A and
centres it is given are the problem's own, and the shape of the A gradient it returns."""
import numpy as np
import pytest
import torch

from paper_1605_01799_amd import hopf as H


def _fake_problem(A, diagonal=False, centres=None, n=None):
    p = H.Problem.__new__(H.Problem)  # no handle: only the host fields the checks read
    p._handle = None
    p.A = None if A is None else np.asarray(A, np.float64)
    p.n = n if n is not None else p.A.shape[0]
    p.diagonal = diagonal or A is None
    p.centres = None if centres is None else np.asarray(centres, np.float64)
    p.K = 1 if centres is None else p.centres.shape[0]
    return p


def test_held_matrices_accepted():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(6, 6))
    A = A @ A.T + 6 * np.eye(6)
    C = rng.normal(size=(3, 6))
    p = _fake_problem(A, centres=C)
    H._check_held(p, "A", torch.tensor(A, dtype=torch.float32))   # FP32 rounding of the same values
    H._check_held(p, "A", torch.tensor(A, dtype=torch.float64))
    H._check_held(p, "centres", torch.tensor(C, dtype=torch.float32))
    H._check_held(p, "A", None)


def test_other_matrices_rejected():
    rng = np.random.default_rng(6)
    A = rng.normal(size=(5, 5))
    A = A @ A.T + 5 * np.eye(5)
    C = rng.normal(size=(2, 5))
    p = _fake_problem(A, centres=C)
    B = A.copy()
    B[1, 2] += 1e-3
    B[2, 1] += 1e-3
    with pytest.raises(ValueError, match="differs"):
        H._check_held(p, "A", torch.tensor(B))
    with pytest.raises(ValueError, match="shape"):
        H._check_held(p, "A", torch.tensor(A[:4, :4]))
    with pytest.raises(ValueError, match="differs"):
        H._check_held(p, "centres", torch.tensor(C + 1.0))
    with pytest.raises(TypeError):
        H._check_held(p, "A", A)


def test_diagonal_and_identity_forms():
    d = np.array([1.0, 2.0, 3.0])
    p = _fake_problem(d, diagonal=True)
    H._check_held(p, "A", torch.tensor(d))                 # the diagonal as a vector
    H._check_held(p, "A", torch.tensor(np.diag(d)))        # or as the full matrix
    with pytest.raises(ValueError):
        H._check_held(p, "A", torch.tensor(np.diag(d) + 0.1))
    q = _fake_problem(None, n=4)
    H._check_held(q, "A", torch.eye(4, dtype=torch.float64))
    H._check_held(q, "A", torch.ones(4))
    H._check_held(q, "centres", torch.zeros(1, 4))
    with pytest.raises(ValueError):
        H._check_held(q, "A", 2 * torch.eye(4))
