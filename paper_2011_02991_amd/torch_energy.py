"""torch binding of the energy and the natural-gradient update (marshalling only).

``energy(ctx, circ, theta)`` is a ``torch.autograd.Function``:

* forward: E(theta) = Re <psi|H|psi> with psi = U(theta)|in>, computed by the
  library (``qng_energy_dev``), which also leaves the final state psi in a
  device buffer kept for the backward pass;
* backward: dE/dtheta by the library's reverse sweep from that final state
  (``qng_energy_grad_from_state_dev``): two registers swept once through the
  adjoint gates, one Pauli-weighted inner product per parameter (O(P) gates,
  O(1) states), the gradient of the energy defined in Sec. 1 of the paper.

``NaturalGradient`` applies the paper's update (Sec. 1): with g = Re G,
(g + eps I) dtheta = -dt dE/dtheta, G recomputed by the recurrent metric
(``qng_metric``) at the current theta and the shifted system solved by the
library's FP64 Cholesky (``qng_solve_shifted``).

All library calls run on torch's current stream of the tensor's device.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import Circuit, Context, solve_shifted


def _bind_stream(qctx: Context, device: torch.device) -> None:
    s = torch.cuda.current_stream(device)
    qctx.set_stream(s.cuda_stream or None)


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, qctx: Context, circ: Circuit, prec: str, in_state: Optional[torch.Tensor]):
        if theta.dim() != 1 or theta.shape[0] != circ.n_params:
            raise ValueError(f"theta must have shape ({circ.n_params},)")
        dev = in_state.device if in_state is not None else torch.device("cuda", torch.cuda.current_device())
        if dev.type != "cuda":
            raise ValueError("in_state must be a CUDA tensor")
        _bind_stream(qctx, dev)
        th = theta.detach().to("cpu", torch.float64).numpy().copy()
        E = torch.empty((), dtype=torch.float64, device=dev)
        psi = torch.empty(2 ** circ.n_qubits, dtype=torch.complex128, device=dev)
        ins = None
        if in_state is not None:
            if in_state.dtype != torch.complex128 or not in_state.is_contiguous():
                raise ValueError("in_state must be a contiguous complex128 tensor")
            ins = in_state.data_ptr()
        qctx.energy_dev(circ, th, E.data_ptr(), psi.data_ptr(), in_state_dev_ptr=ins, prec=prec)
        fctx.qctx, fctx.circ, fctx.prec, fctx.th = qctx, circ, prec, th
        fctx.psi = psi
        fctx.theta_meta = (theta.device, theta.dtype)
        return E.to(theta.dtype) if theta.dtype != torch.float64 else E

    @staticmethod
    def backward(fctx, gE: torch.Tensor):
        psi = fctx.psi
        _bind_stream(fctx.qctx, psi.device)
        grad = torch.empty(fctx.circ.n_params, dtype=torch.float64, device=psi.device)
        fctx.qctx.energy_grad_from_state_dev(fctx.circ, fctx.th, psi.data_ptr(), grad.data_ptr(), prec=fctx.prec)
        fctx.psi = None
        device, dtype = fctx.theta_meta
        g = (gE.to(torch.float64) * grad).to(device=device, dtype=dtype)
        return g, None, None, None, None


def energy(qctx: Context, circ: Circuit, theta: torch.Tensor, prec: str = "c128",
           in_state: Optional[torch.Tensor] = None) -> torch.Tensor:
    """E(theta) as a differentiable scalar (see the module docstring).  theta may
    live on the host or the device; the gradient comes back on its device."""
    if circ.h is None:
        raise ValueError("circuit has no Hamiltonian")
    return _Energy.apply(theta, qctx, circ, prec, in_state)


class NaturalGradient:
    """theta <- theta + dtheta with (Re G + eps I) dtheta = -dt grad, where grad
    is theta.grad (filled by a backward pass of ``energy``)."""

    def __init__(self, qctx: Context, circ: Circuit, theta: torch.Tensor, dt: float, tikhonov: float = 1e-4,
                 prec: str = "c128", in_state: Optional[np.ndarray] = None):
        self.qctx, self.circ, self.theta = qctx, circ, theta
        self.dt, self.tikhonov, self.prec, self.in_state = float(dt), float(tikhonov), prec, in_state
        self.last_G = None

    @torch.no_grad()
    def step(self) -> np.ndarray:
        if self.theta.grad is None:
            raise RuntimeError("theta.grad is empty: call backward() on the energy first")
        th = self.theta.detach().to("cpu", torch.float64).numpy()
        grad = self.theta.grad.detach().to("cpu", torch.float64).numpy()
        G, _ = self.qctx.metric(self.circ, th, in_state=self.in_state, prec=self.prec)
        dtheta = solve_shifted(G, self.tikhonov, -self.dt * grad)
        self.theta.add_(torch.as_tensor(dtheta, dtype=self.theta.dtype).to(self.theta.device))
        self.last_G = G
        return dtheta

    def zero_grad(self):
        self.theta.grad = None
