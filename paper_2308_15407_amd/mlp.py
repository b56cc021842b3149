"""WarmStartNet: the multilayer perceptron of the learned warm start, run and
trained by libfdlb's own kernels (BF16 MFMA GEMMs, GELU, MSE, AdamW).

Layout of the flat parameter vector: for each layer W[out][in] row-major then
b[out].  Initial weights are drawn on the host from a seeded generator and
passed in (uniform +-sqrt(6/fan_in) for W, zeros for b).
"""
import numpy as np
import torch

from . import fdlb as F


def layer_shapes(n_in, width, depth, n_out):
    dims = [n_in] + [width] * depth + [n_out]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def init_params(n_in, width, depth, n_out, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fin, fout in layer_shapes(n_in, width, depth, n_out):
        lim = np.sqrt(6.0 / fin)
        parts.append(rng.uniform(-lim, lim, size=(fout, fin)).astype(np.float32).ravel())
        parts.append(np.zeros(fout, dtype=np.float32))
    return np.concatenate(parts)


class WarmStartNet:
    def __init__(self, n_in=10, width=256, depth=4, n_out=640, max_batch=4096, device="cuda:0", seed=0):
        if not torch.cuda.is_available():
            raise RuntimeError("WarmStartNet needs a HIP device")
        self.n_in, self.width, self.depth, self.n_out, self.max_batch = n_in, width, depth, n_out, max_batch
        self.device = torch.device(device)
        nb = F.fdlb_mlp_workspace_bytes(n_in, width, depth, n_out, max_batch)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = F.fdlb_mlp_init(n_in, width, depth, n_out, max_batch, self.workspace.data_ptr(), nb,
                                      self.stream.cuda_stream)
        self.nparams = F.fdlb_mlp_num_params(self.handle)
        self.set_params(init_params(n_in, width, depth, n_out, seed))

    def close(self):
        if getattr(self, "handle", None):
            F.fdlb_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        assert p.size == self.nparams
        F.fdlb_mlp_set_params(self.handle, p)

    def get_params(self):
        return F.fdlb_mlp_get_params(self.handle, self.nparams)

    def _dev(self, a, cols):
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)) if not torch.is_tensor(a) else a
        t = t.to(self.device, dtype=torch.float32).contiguous()
        assert t.dim() == 2 and t.shape[1] == cols and t.shape[0] <= self.max_batch
        return t

    def forward(self, x):
        x = self._dev(x, self.n_in)
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=self.device)
        F.fdlb_mlp_forward(self.handle, x.data_ptr(), x.shape[0], y.data_ptr())
        return y

    def loss_grad(self, x, t):
        x, t = self._dev(x, self.n_in), self._dev(t, self.n_out)
        return F.fdlb_mlp_loss_grad(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], self.nparams)

    def train_step(self, x, t, lr, weight_decay=0.0, want_loss=False):
        x, t = self._dev(x, self.n_in), self._dev(t, self.n_out)
        return F.fdlb_mlp_train_step(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0], lr, weight_decay, want_loss)
