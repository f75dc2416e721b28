"""torch.autograd bridge of qsv_expval_grad (argument marshalling only).

The paper's variational workflow binds a compiled program's ``input`` angles
at run time, many times over (Background: parameter passing and VQE;
Methodology: handling runtime parameters). Here the energies E_b = <psi(theta_b)|
H |psi(theta_b)> of a batch of parameter vectors are a differentiable torch
function of theta: the forward pass calls qsv_expval_grad once with device
pointers ordered on the context's stream, which returns the energies and the
adjoint gradients together; the backward pass only scales the stored gradient
rows by the incoming gradient of each energy.

The context must be created with ``device_ptrs=True`` and with torch's current
stream as its stream (``Context(dev, stream=torch.cuda.current_stream(),
device_ptrs=True)``), so the library reads theta and writes its outputs in
torch's stream order; theta is a float64 CUDA tensor [B, P] (or [P]).
"""
import torch

from .api import QsvError


class _Expval(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, prog, hamiltonian):
        b, p = theta.shape
        energy = torch.empty(b, dtype=torch.float64, device=theta.device)
        grad = torch.empty((b, max(1, p)), dtype=torch.float64, device=theta.device)
        prog.expval_grad_device(theta.data_ptr(), b, hamiltonian, energy.data_ptr(), grad.data_ptr())
        fctx.save_for_backward(grad[:, :p])
        return energy

    @staticmethod
    def backward(fctx, g_energy):
        (grad,) = fctx.saved_tensors
        return g_energy.to(grad.dtype)[:, None] * grad, None, None


def expval(prog, theta, coeffs, codes):
    """Differentiable energies of `prog` (a unitary qsv Program) for theta [B, P]
    or [P] (float64 CUDA tensor) under H = sum_j coeffs[j] P_j (codes[j][q] in
    0..3 = I, X, Y, Z). Returns [B] (or a scalar for a 1-D theta)."""
    ctx = prog.ctx
    if not ctx.device_ptrs:
        raise QsvError(-1, "the context must be created with device_ptrs=True")
    cur = torch.cuda.current_stream(theta.device).cuda_stream
    if ctx.stream_handle != cur:
        raise QsvError(-1, "the context's stream must be torch's current stream on theta's device")
    if theta.dtype != torch.float64 or not theta.is_cuda:
        raise TypeError("theta must be a float64 CUDA tensor")
    squeeze = theta.dim() == 1
    t = theta.reshape(1, -1) if squeeze else theta
    if t.shape[1] != prog.info.n_params:
        raise ValueError(f"theta must hold {prog.info.n_params} values per vector")
    h, keep = prog._pauli(coeffs, codes)
    e = _Expval.apply(t.contiguous(), prog, h)
    del keep
    return e[0] if squeeze else e
