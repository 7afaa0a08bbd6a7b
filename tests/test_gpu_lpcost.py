"""GPU parity of the differentiable cost (forward + hand-written backward)
against the float64 oracle, which the CPU tests pin to central differences
and to torch's float64 autograd."""
import numpy as np
import pytest

from gpu_common import say
from oracle import prost_oracle as O
from synth import video as V

pytestmark = pytest.mark.gpu

TOL = 1e-4   # relative, per tensor (Frobenius)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _run(U, Y, X, w, mu, p, cost, gout):
    import torch
    from paper_1302_2073_amd.lpcost import lpcost
    dev = "cuda"
    tU = torch.tensor(U, dtype=torch.float32, device=dev, requires_grad=True)
    tY = torch.tensor(Y.T.copy(), dtype=torch.float32, device=dev, requires_grad=True)   # (B, k)
    tX = torch.tensor(X.T.copy(), dtype=torch.float32, device=dev, requires_grad=True)   # (B, m)
    tmu = torch.tensor([mu], dtype=torch.float32, device=dev, requires_grad=True)
    tw = None if w is None else torch.tensor(w, dtype=torch.float32, device=dev)
    f = lpcost(tU, tY, tX, tmu, tw, p, cost)
    f.backward(torch.tensor(gout, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    return (f.detach().cpu().numpy().astype(np.float64), tU.grad.cpu().numpy().astype(np.float64),
            tY.grad.cpu().numpy().T.astype(np.float64), tX.grad.cpu().numpy().T.astype(np.float64),
            float(tmu.grad.item()))


def _oracle(U, Y, X, w, mu, p, cost, gout):
    U64, Y64, X64 = (np.asarray(a, np.float32).astype(np.float64) for a in (U, Y, X))
    w64 = np.ones(U.shape[0]) if w is None else np.asarray(w, np.float32).astype(np.float64)
    mu64 = float(np.float32(mu))
    g64 = np.asarray(gout, np.float32).astype(np.float64)
    f = O.lpcost_forward(U64, Y64, X64, w64, p, mu64, cost)
    dX, dU, dY, dmu = O.lpcost_backward(U64, Y64, X64, w64, p, mu64, g64, cost)
    return f, dU, dY, dX, dmu


def _check(args, label):
    got = _run(*args)
    exp = _oracle(*args)
    errs = [_rel(g, e) for g, e in zip(got[:4], exp[:4])] + [abs(got[4] - exp[4]) / abs(exp[4])]
    say(f"  {label}: f {errs[0]:.1e} dU {errs[1]:.1e} dY {errs[2]:.1e} dX {errs[3]:.1e} dmu {errs[4]:.1e}")
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("cost,p", [("lp", 0.25), ("log", 0.25), ("lp", 1.0)])
@pytest.mark.parametrize("shape", [(1000, 5, 3), (777, 16, 1), (5000, 1, 70), (3001, 10, 33)])
@pytest.mark.parametrize("weighted", [False, True])
def test_small(shape, cost, p, weighted):
    m, k, B = shape
    rng = np.random.default_rng([m, k, B])
    U = V.random_orthonormal(m, k, rng)
    Y = 0.3 * rng.standard_normal((k, B))
    X = U @ Y + 0.05 * rng.standard_normal((m, B))
    X[rng.random((m, B)) < 0.1] = 0.7
    w = np.where(rng.random(m) < 0.2, 5e-5, 1.0) if weighted else None
    gout = rng.standard_normal(B)
    _check((U, Y, X, w, 1e-3, p, cost, gout), f"m={m} k={k} B={B} {cost} p={p} w={weighted}")


@pytest.mark.parametrize("weighted", [False, True])
def test_full_size_320x240x3_k10_b32(weighted):
    """The differentiation workload: m = 230400, k = 10, B = 32."""
    U, Y, X, w = V.lpcost_batch(weighted=weighted)
    gout = np.random.default_rng(9).standard_normal(32)
    _check((U, Y, X, w if weighted else None, 1e-3, 0.25, "lp", gout), f"full weighted={weighted}")


def test_single_frame_du_is_eta_y():
    """B = 1, upstream gradient 1: dU = eta y^T of Sec. 3.3 (Step 2)."""
    rng = np.random.default_rng(3)
    m, k = 4000, 6
    U = V.random_orthonormal(m, k, rng)
    y = rng.standard_normal(k) * 0.2
    x = U @ y + 0.02 * rng.standard_normal(m)
    w = np.where(rng.random(m) < 0.1, 5e-5, 1.0)
    f, dU, dY, dX, dmu = _run(U, y[:, None], x[:, None], w, 1e-3, 0.25, "lp", np.ones(1))
    U64, y64, x64, w64 = (np.asarray(a, np.float32).astype(np.float64) for a in (U, y, x, w))
    eta = O.eta_vector(U64, x64, y64, w64, 0.25, float(np.float32(1e-3)))
    assert _rel(dU, np.outer(eta, y64)) <= TOL
