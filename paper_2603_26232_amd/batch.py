"""Torch-facing wrapper of the batch ABI: PyTorch supplies device memory and
the stream, every computation runs in libparaqaoa's HIP kernels."""
from __future__ import annotations

import numpy as np
import torch

from . import _abi
from .partition import batch_arrays


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class QaoaBatch:
    """A batch of subgraphs on one GPU (states, cut tables, phase tables in
    one caller-owned workspace tensor)."""

    MIXERS = {"valu": 0, "mfma_f32": _abi.QAOA_FLAG_MIXER_MFMA_F32, "mfma_bf16x3": _abi.QAOA_FLAG_MIXER_MFMA_BF16X3,
              "mfma_bf16x4": _abi.QAOA_FLAG_MIXER_MFMA_BF16X4}
    # gradient memory: the library's choice, forward checkpoints, or one psi rebuilt in place
    GRADIENT_MEMORY = {"auto": 0, "checkpoints": _abi.QAOA_FLAG_GRADIENT_CHECKPOINTS,
                       "inplace": _abi.QAOA_FLAG_GRADIENT_INPLACE}

    def __init__(self, sizes, sub_edges, max_p, max_k=16, gradient=False, raw_topk=False,
                 skip_edgeless=False, device="cuda", stream=None, mixer="valu", gradient_memory="auto",
                 concurrent_classes=False):
        nq, off, u, v, w = batch_arrays(sizes, sub_edges)
        self.B = int(nq.shape[0])
        self.sizes = nq
        self.max_p = int(max_p)
        self.max_k = int(max_k)
        self.device = torch.device(device)
        flags = ((_abi.QAOA_FLAG_GRADIENT if gradient else 0) | (_abi.QAOA_FLAG_TOPK_RAW if raw_topk else 0)
                 | (_abi.QAOA_FLAG_SKIP_EDGELESS if skip_edgeless else 0) | self.MIXERS[mixer]
                 | self.GRADIENT_MEMORY[gradient_memory]
                 | (_abi.QAOA_FLAG_CONCURRENT_CLASSES if concurrent_classes else 0))
        self.flags = flags
        nbytes = _abi.qaoa_workspace_bytes(self.B, nq, off, w, self.max_p, self.max_k, flags)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = _abi.qaoa_batch_create(self.B, nq, off, u, v, w, self.max_p, self.max_k, flags,
                                             _ptr(self.workspace), nbytes, _stream(stream))

    def close(self):
        if getattr(self, "handle", 0):
            _abi.qaoa_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _angles(a, device):
        return torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()

    def apply_layers(self, gamma, beta, stream=None):
        g = self._angles(gamma, self.device)
        b = self._angles(beta, self.device)
        p = g.numel() // self.B
        _abi.qaoa_apply_layers(self.handle, p, _ptr(g), _ptr(b), _stream(stream))
        self._keep = (g, b)

    def expectation(self, out=None, stream=None):
        out = torch.empty(self.B, dtype=torch.float64, device=self.device) if out is None else out
        _abi.qaoa_expectation(self.handle, _ptr(out), _stream(stream))
        return out

    def topk(self, k, stream=None):
        idx = torch.empty(self.B * k, dtype=torch.int32, device=self.device)
        prob = torch.empty(self.B * k, dtype=torch.float32, device=self.device)
        _abi.qaoa_topk(self.handle, k, _ptr(idx), _ptr(prob), _stream(stream))
        return idx.view(self.B, k), prob.view(self.B, k)

    def expectation_grad(self, gamma, beta, E=None, dgamma=None, dbeta=None, stream=None):
        g = self._angles(gamma, self.device)
        b = self._angles(beta, self.device)
        p = g.numel() // self.B
        E = torch.empty(self.B, dtype=torch.float64, device=self.device) if E is None else E
        dg = torch.empty(self.B * p, dtype=torch.float64, device=self.device) if dgamma is None else dgamma
        db = torch.empty(self.B * p, dtype=torch.float64, device=self.device) if dbeta is None else dbeta
        _abi.qaoa_expectation_grad(self.handle, p, _ptr(g), _ptr(b), _ptr(E), _ptr(dg), _ptr(db),
                                   _stream(stream))
        return E, dg.view(self.B, p), db.view(self.B, p)

    def reduced_state(self, b: int) -> torch.Tensor:
        """View of subgraph b's stored state inside the workspace: the 2^(n-1)
        amplitudes with the top bit clear, scaled by sqrt(2) (unit norm)."""
        off = _abi.qaoa_state_offset(self.handle, b)
        n = int(self.sizes[b])
        return self.workspace[off:off + 8 * (1 << (n - 1))].view(torch.complex64)

    def state(self, b: int) -> torch.Tensor:
        """Subgraph b's full complex64 state (a new tensor): psi(z) =
        phi(z) / sqrt(2) for z < 2^(n-1), and psi(z) = psi(complement of z),
        i.e. the upper half is the lower half reversed."""
        phi = self.reduced_state(b)
        return torch.cat([phi, phi.flip(0)]) * (2.0 ** -0.5)


def idx_to_uint32(idx: torch.Tensor) -> np.ndarray:
    return idx.cpu().numpy().view(np.uint32)
