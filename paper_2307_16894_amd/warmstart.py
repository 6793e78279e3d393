"""Learned Newton warm start: sample generation with the library's FP64
solve and training with the library's own network kernels.

Samples are (features, dr) pairs of converged load steps: rom_features gives
the inputs for the step (mu, Fbar - Fbar_committed, r_committed, eight plastic
statistics), and rom_warm_samples appends the converged points' features and
dr = r_converged - r_committed.  The scaling is fitted by rom_mlp_fit_scaling,
and rom_mlp_train_epoch runs the minibatches (gathering their rows itself).
Python only allocates buffers, draws the per-epoch permutation of the sample
indices (a seeded generator) and the learning-rate schedule, and marshals
arguments: the arithmetic runs in libpodecm.
"""
import numpy as np
import torch

from . import (DT_BF16, DT_F64, MODE_FUSED, WARM_MLP, rom_default_opts, rom_features, rom_mlp_create,
               rom_mlp_fit_scaling, rom_mlp_free, rom_mlp_get_params, rom_mlp_param_count, rom_mlp_set_params,
               rom_mlp_train_epoch, rom_state_init, rom_warm_samples)

WIDTH = 256


def init_params(n_in, width, n_out, seed):
    """Uniform fan-in initialisation, flat in the library's parameter layout."""
    g = np.random.Generator(np.random.PCG64(seed))
    dims = [n_in, width, width, width, n_out]
    out = []
    for l, (fi, fo) in enumerate(zip(dims[:-1], dims[1:])):
        lim = np.sqrt(6.0 / fi) * (0.5 if l == 3 else 1.0)
        out.append(g.uniform(-lim, lim, size=fi * fo))
        out.append(np.zeros(fo))
    return np.concatenate(out).astype(np.float32)


def generate(rb, paths, opts=None):
    """Run every point of RomBatch `rb` along `paths` ((P, K, 2, 2) array) with
    plain FP64 Newton from the virgin state; return device tensors X (samples,
    n_in) and Y (samples, n) of the converged steps."""
    P, K = paths.shape[0], paths.shape[1]
    n, n_mu = rb.info['n'], rb.info['n_mu']
    nf = n_mu + 4 + n + 8
    dev = rb.device
    o = opts if opts is not None else rom_default_opts(mode=MODE_FUSED, contraction=DT_F64)
    rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
    Fb = torch.from_numpy(np.ascontiguousarray(paths.reshape(P, K, 4).transpose(1, 0, 2))).to(dev)
    X = torch.empty(P, nf, dtype=torch.float32, device=dev)
    r0 = torch.empty(P, n, dtype=torch.float64, device=dev)
    Xs = torch.empty(P * K, nf, dtype=torch.float32, device=dev)
    Ys = torch.empty(P * K, n, dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    s = rb.stream.cuda_stream
    for k in range(K):
        rom_features(rb.h, P, Fb[k].data_ptr(), rb.state.data_ptr(), X.data_ptr(), s)
        r0.copy_(rb.r())
        rb.step(Fb[k], o)
        rom_warm_samples(rb.h, P, rb.state.data_ptr(), X.data_ptr(), r0.data_ptr(), rb.status.data_ptr(),
                         Xs.data_ptr(), Ys.data_ptr(), count.data_ptr(), s)
    N = int(count.item())
    return Xs[:N], Ys[:N]


class WarmStart:
    """Owns a library network; trains it on (X, Y) device tensors."""

    def __init__(self, n_in, n_out, width=WIDTH, max_batch=4096, device=0, seed=0):
        self.n_in, self.n_out, self.width = n_in, n_out, width
        self.h = rom_mlp_create(n_in, width, n_out, max_batch, device)
        self.max_batch = max_batch
        rom_mlp_set_params(self.h, init_params(n_in, width, n_out, seed))

    def close(self):
        if self.h is not None:
            rom_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self):
        return rom_mlp_param_count(self.h)

    def params(self):
        return rom_mlp_get_params(self.h)

    def fit_scaling(self, X, Y):
        rom_mlp_fit_scaling(self.h, X.shape[0], X.contiguous().data_ptr(), Y.contiguous().data_ptr(),
                            torch.cuda.current_stream(X.device).cuda_stream)

    def train(self, X, Y, epochs=10, batch=1024, lr=1e-3, precision=DT_BF16, seed=0, stream=None, log=None):
        """Minibatch Adam with a cosine-decayed learning rate; the samples are
        visited in a fresh seeded permutation each epoch.  Returns the mean
        loss of each epoch."""
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        g = np.random.Generator(np.random.PCG64(seed))
        N = X.shape[0]
        batch = min(batch, self.max_batch)
        nb = N // batch
        X, Y = X.contiguous(), Y.contiguous()
        order = torch.empty(N, dtype=torch.int32, device=X.device)
        sums = torch.zeros(epochs, dtype=torch.float32, device=X.device)
        for e in range(epochs):
            with torch.cuda.stream(s):  # ordered after the previous epoch's reads of `order`
                order.copy_(torch.from_numpy(g.permutation(N).astype(np.int32)))
            lr_e = lr * 0.5 * (1.0 + np.cos(np.pi * e / max(epochs, 1)))
            rom_mlp_train_epoch(self.h, N, X.data_ptr(), Y.data_ptr(), order.data_ptr(), batch, max(lr_e, 1e-6),
                                precision, sums[e:e + 1].data_ptr(), s.cuda_stream)
            if log:
                log(f"epoch {e}: loss {float(sums[e]) / max(nb, 1):.4e}")
        return [float(v) / max(nb, 1) for v in sums.cpu().numpy()]

    def opts(self, **kw):
        kw.setdefault('mode', MODE_FUSED)
        o = rom_default_opts(warm_start=WARM_MLP, **kw)
        o.mlp = self.h.value
        return o
