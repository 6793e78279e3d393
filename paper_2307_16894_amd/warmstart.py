"""Learned Newton warm start: sample generation with the library's FP64
solve and training with the library's own network kernels.

Samples are (features, dr) pairs of converged load steps: rom_features gives
the inputs for the step (mu, Fbar - Fbar_committed, r_committed, eight plastic
statistics) and dr = r_converged - r_committed is the target.  Python only
marshals arguments and shuffles sample indices; the network's forward,
backward and Adam updates run in libpodecm.
"""
import numpy as np
import torch

from . import (DT_BF16, DT_F64, MODE_FUSED, WARM_MLP, rom_default_opts, rom_features, rom_mlp_create,
               rom_mlp_free, rom_mlp_get_params, rom_mlp_param_count, rom_mlp_set_params, rom_mlp_set_scaling,
               rom_mlp_train_step, rom_state_init)

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
    Xs, Ys = [], []
    X = torch.empty(P, nf, dtype=torch.float32, device=dev)
    for k in range(K):
        rom_features(rb.h, P, Fb[k].data_ptr(), rb.state.data_ptr(), X.data_ptr(), rb.stream.cuda_stream)
        r0 = rb.r().clone()
        rb.step(Fb[k], o)
        ok = rb.status == 0
        Xs.append(X[ok].clone())
        Ys.append((rb.r() - r0)[ok].float())
    return torch.cat(Xs), torch.cat(Ys)


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
        xm = X.mean(0).cpu().numpy()
        xs = X.std(0).cpu().numpy()
        ym = Y.mean(0).cpu().numpy()
        ys = Y.std(0).cpu().numpy()
        xs = np.where(xs > 1e-12, xs, 1.0)
        ys = np.where(ys > 1e-12, ys, 1.0)
        rom_mlp_set_scaling(self.h, xm, xs, ym, ys)

    def train(self, X, Y, epochs=10, batch=1024, lr=1e-3, precision=DT_BF16, seed=0, stream=None, log=None):
        """Minibatch Adam; returns the mean loss of each epoch."""
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        g = torch.Generator(device=X.device)
        g.manual_seed(seed)
        N = X.shape[0]
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        hist = []
        batch = min(batch, self.max_batch)
        for e in range(epochs):
            perm = torch.randperm(N, generator=g, device=X.device)
            tot = torch.zeros((), dtype=torch.float32, device=X.device)
            nb = 0
            # cosine decay of the learning rate over the epochs
            lr_e = lr * 0.5 * (1.0 + np.cos(np.pi * e / max(epochs, 1)))
            for b0 in range(0, N - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                xb = X[idx].contiguous()
                yb = Y[idx].contiguous()
                rom_mlp_train_step(self.h, batch, xb.data_ptr(), yb.data_ptr(), max(lr_e, 1e-6), precision,
                                   loss.data_ptr(), s.cuda_stream)
                tot += loss[0]
                nb += 1
            hist.append(float(tot) / max(nb, 1))
            if log:
                log(f"epoch {e}: loss {hist[-1]:.4e}")
        return hist

    def opts(self, **kw):
        kw.setdefault('mode', MODE_FUSED)
        o = rom_default_opts(warm_start=WARM_MLP, **kw)
        o.mlp = self.h.value
        return o
