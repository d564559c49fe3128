"""Gradient conventions of the autograd wrappers, on the CPU with a dense
stand-in operator: the wrappers' backward (adjoint call) must agree with
PyTorch's own autograd through the explicit matrix A = exp(-2 pi i P R^T)."""
import numpy as np
import torch

from paper_2306_06007_amd.autograd import HvoxAnalysis, HvoxSynthesis


class DensePlan:
    complex_dtype = torch.complex128

    def __init__(self, P, R):
        self.A = torch.as_tensor(np.exp(-2j * np.pi * (P @ R.T)))

    def synthesis(self, x):
        return (self.A @ x.T).T

    def analysis(self, v):
        return (self.A.conj().T @ v.T).T


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    P = rng.uniform(-50, 50, (30, 3))
    R = rng.normal(size=(20, 3))
    return DensePlan(P, R), rng


def test_real_input_gradient_matches_dense_autograd():
    plan, rng = _setup()
    y = torch.as_tensor(rng.normal(size=(1, 30)) + 1j * rng.normal(size=(1, 30)))
    x0 = rng.random((1, 20))
    x = torch.tensor(x0, requires_grad=True)
    V = HvoxSynthesis.apply(x, plan)
    (0.5 * (V - y).abs().pow(2).sum()).backward()
    xr = torch.tensor(x0, requires_grad=True)
    Vr = (plan.A @ xr.to(torch.complex128).T).T
    (0.5 * (Vr - y).abs().pow(2).sum()).backward()
    assert torch.allclose(x.grad, xr.grad, rtol=1e-12, atol=1e-12)
    # closed form: Re(A^H (A x - y))
    closed = (plan.A.conj().T @ (Vr.detach() - y).T).T.real
    assert torch.allclose(x.grad, closed, rtol=1e-12, atol=1e-12)


def test_complex_input_and_analysis_gradients():
    plan, rng = _setup(1)
    x0 = rng.normal(size=(2, 20)) + 1j * rng.normal(size=(2, 20))
    w = torch.as_tensor(rng.normal(size=(2, 30)) + 1j * rng.normal(size=(2, 30)))
    x = torch.tensor(x0, requires_grad=True)
    (HvoxSynthesis.apply(x, plan) * w.conj()).real.sum().backward()
    xr = torch.tensor(x0, requires_grad=True)
    ((plan.A @ xr.T).T * w.conj()).real.sum().backward()
    assert torch.allclose(x.grad, xr.grad, rtol=1e-12, atol=1e-12)
    v0 = rng.normal(size=(1, 30)) + 1j * rng.normal(size=(1, 30))
    v = torch.tensor(v0, requires_grad=True)
    HvoxAnalysis.apply(v, plan).abs().pow(2).sum().backward()
    vr = torch.tensor(v0, requires_grad=True)
    (plan.A.conj().T @ vr.T).T.abs().pow(2).sum().backward()
    assert torch.allclose(v.grad, vr.grad, rtol=1e-12, atol=1e-12)
