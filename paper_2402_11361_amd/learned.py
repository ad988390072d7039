"""Learned coarse correction for the FGMRES preconditioner: harvesting of
training pairs from the method's own solves, training on the GPU through the
library's kernels, and binding of the trained network (BF16) to the solver.

FGMRES (Sec. 4.2) accepts a preconditioner that varies between steps; the
learned stage adds P_c f(R_c v) to the plain preconditioner z_p = P(v), with
f trained to map the coarse coefficients R_c v of a vector to those of
A-hat^{-1} v - z_p, i.e. the coarse part of what the plain stage misses.
Host code here only orders the calls; all arithmetic runs in libhdg.so.
"""
import ctypes

import numpy as np

from .hdg import HDG_FP64, Mlp


class CoarseCorrection:
    def __init__(self, ctx, hidden=256, max_batch=1024, seed=0, neighbours=False):
        """neighbours: the network also sees the coarse coefficients of the
        macros across each face (hdg_coarse_neighbours), (1 + 2d) F inputs."""
        import torch
        self.t = torch
        self.ctx = ctx
        F = ctx.coarse_size()
        self.neighbours = bool(neighbours)
        n_in = (1 + 2 * ctx.dim) * F if self.neighbours else F
        self.F, self.n_in, self.hidden, self.max_batch = F, n_in, hidden, max_batch
        lib = ctx.lib
        n = int(lib.hdg_mlp_param_count(n_in, hidden, F))
        nw = int(lib.hdg_mlp_work_floats(n_in, hidden, F, max_batch))
        # Glorot-uniform weights, zero biases, from a seeded host generator
        rng = np.random.default_rng(seed)
        a1 = np.sqrt(6.0 / (n_in + hidden))
        a2 = np.sqrt(6.0 / (hidden + F))
        p0 = np.concatenate([rng.uniform(-a1, a1, hidden * n_in), np.zeros(hidden),
                             rng.uniform(-a2, a2, F * hidden), np.zeros(F)]).astype(np.float32)
        assert p0.size == n
        dev = dict(dtype=torch.float32, device="cuda")
        self.params = torch.tensor(p0, **dev)
        self.grads = torch.zeros(n, **dev)
        self.adam_m = torch.zeros(n, **dev)
        self.adam_v = torch.zeros(n, **dev)
        self.work = torch.zeros(nw, **dev)
        self.loss = torch.zeros(1, **dev)
        self.net = Mlp(n_in, hidden, F, max_batch, self.params.data_ptr(), self.grads.data_ptr(),
                       self.adam_m.data_ptr(), self.adam_v.data_ptr(), self.work.data_ptr())
        self.X, self.T = [], []
        self.step = 0

    # ---- data -----------------------------------------------------------------
    def harvest(self, bhat, n_vectors=40, rtol=1e-8, target_rtol=1e-6, restart=30, inner_its=5,
                inner_prec=HDG_FP64):
        """Pairs (R_c v, R_c (A-hat^{-1} v - P(v))) for the first n_vectors
        vectors v that a plain FGMRES solve of A-hat x = bhat preconditions
        (needs a condensed operator)."""
        t, ctx = self.t, self.ctx
        H = t.empty(n_vectors, ctx.n_glob, dtype=t.float64, device="cuda")
        x = t.zeros(ctx.n_glob, dtype=t.float64, device="cuda")
        info = ctx.fgmres_solve(bhat, x, rtol=rtol, restart=restart, inner_its=inner_its, inner_prec=inner_prec,
                                harvest=H, allow_noconv=True)
        k = info["harvested"]
        e = t.empty(ctx.n_glob, dtype=t.float64, device="cuda")
        zp = t.empty_like(e)
        for j in range(k):
            v = H[j]
            e.zero_()
            ctx.fgmres_solve(v, e, rtol=target_rtol, restart=restart, inner_its=inner_its, inner_prec=inner_prec,
                             allow_noconv=True)
            ctx.precond_apply(v, zp, inner_its, inner_prec)
            ctx.axpy(-1.0, zp, e)  # e = A-hat^{-1} v - P(v)
            Xj = t.empty(ctx.n_macros, self.F, dtype=t.float32, device="cuda")
            Tj = t.empty_like(Xj)
            ctx.coarse_restrict(v, Xj)
            ctx.coarse_restrict(e, Tj)
            if self.neighbours:
                Xe = t.empty(ctx.n_macros, self.n_in, dtype=t.float32, device="cuda")
                ctx.coarse_neighbours(Xj, Xe)
                Xj = Xe
            self.X.append(Xj)
            self.T.append(Tj)
        return k

    def n_pairs(self):
        return sum(x.shape[0] for x in self.X)

    # ---- training -------------------------------------------------------------
    def train(self, epochs=100, lr=1e-3, batch=None, seed=0, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam on the mean squared error in normalised units; returns the mean
        loss of each epoch."""
        t, ctx = self.t, self.ctx
        X = t.cat(self.X).contiguous()
        T = t.cat(self.T).contiguous()
        N = X.shape[0]
        B = min(batch or self.max_batch, self.max_batch, N)
        gen = t.Generator(device="cpu")
        gen.manual_seed(seed)
        hist = []
        acc = t.zeros(1, dtype=t.float32, device="cuda")
        for ep in range(epochs):
            perm = t.randperm(N, generator=gen).to(dtype=t.int32, device="cuda")
            acc.zero_()
            nb = N // B
            for b in range(nb):
                idx = perm[b * B:(b + 1) * B]
                ctx.mlp_loss_grad(self.net, X, T, idx, B, self.loss)
                self.step += 1
                ctx.mlp_adam(self.net, lr, beta1, beta2, eps, self.step)
                acc += self.loss
            hist.append(float(acc.item()) / max(nb, 1))
        return hist

    def eval_loss(self, X, T):
        """Loss of the current network on (X, T) in batches."""
        t, ctx = self.t, self.ctx
        N = X.shape[0]
        B = min(self.max_batch, N)
        tot, cnt = 0.0, 0
        for b0 in range(0, N - B + 1, B):
            idx = t.arange(b0, b0 + B, dtype=t.int32, device="cuda")
            ctx.mlp_loss_grad(self.net, X, T, idx, B, self.loss)
            tot += float(self.loss.item())
            cnt += 1
        return tot / max(cnt, 1)

    def bind(self):
        self.ctx.learned_bind(self.net)

    def unbind(self):
        self.ctx.learned_bind(None)

    def params_numpy(self):
        return self.params.cpu().numpy().astype(np.float64)
