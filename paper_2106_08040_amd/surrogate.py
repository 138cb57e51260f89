"""Learned surrogate of the solver: a two-member network ensemble trained on the solver's own
harmonics, evaluated with the solver as fallback (fpn_surrogate_predict).

Everything numeric runs in the library: the solver makes the training targets (fpn_solve), the
features come from fpn_surrogate_features, training steps are fpn_mlp_train_step (BF16 matrix-core
products, FP32 Adam) and prediction is fpn_surrogate_predict.  This module only orders those calls:
it draws minibatch indices, sets the learning-rate schedule and picks the calibration constant of
the error estimate from held-out solver results.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import SurrogateModel

WIDTHS_HIDDEN = (512, 512, 512, 512)


def harm_targets(harm):
    """Network target layout [n, 4 K] = [channel x, y][k = 1..K][re, im] from solver harmonics
    (complex [n, 2, K + 1])."""
    torch = _torch()
    h = torch.view_as_real(harm[:, :2, 1:].contiguous())  # [n, 2, K, 2]
    return h.reshape(h.shape[0], -1).contiguous()


def _torch():
    import torch
    return torch


class Surrogate:
    """Two networks of identical shape, the output scale and the calibrated error constant, held by
    one library model (fpn_sur_model), which can be saved and loaded (``save``, ``Surrogate.load``)."""

    def __init__(self, ctx, n_harm, hidden=WIDTHS_HIDDEN, seeds=(1, 2), model=None):
        self.ctx = ctx
        self.n_harm = int(n_harm)
        widths = [8, *hidden, 4 * self.n_harm]
        self.model = model if model is not None else SurrogateModel(ctx, widths, seeds=seeds)
        if self.model.widths[0] != 8 or self.model.widths[-1] != 4 * self.n_harm:
            raise ValueError("model widths do not map 8 features to 4 * n_harm outputs")
        self.nets = self.model.members
        self.train_seconds = 0.0

    @classmethod
    def load(cls, ctx, path):
        """A surrogate read from a file written by ``save`` (fpn_surrogate_create)."""
        model = SurrogateModel(ctx, path=path)
        return cls(ctx, model.widths[-1] // 4, model=model)

    def save(self, path):
        self.model.save(path)

    @property
    def out_scale(self):
        return self.model.out_scale

    @property
    def err_calib(self):
        return self.model.err_calib

    def close(self):
        self.model.close()

    def fit(self, inst, harm, steps=3000, batch=4096, lr=2e-3, lr_final=2e-5, seed=0, log=None, residual_steps=0):
        """Train both members on (features(inst), harm) with Adam and a cosine learning-rate decay; with
        residual_steps > 0 a second stage (fpn_surrogate_add_residual) is then trained the same way on each
        member's residual, scaled to unit RMS (member k predicts net_k + res_k / res_scale)."""
        torch = _torch()
        x, st = self.ctx.surrogate_features(inst)
        ok = (st == 0) & torch.isfinite(harm.real).all(dim=(1, 2)) & torch.isfinite(harm.imag).all(dim=(1, 2))
        x = x[ok].contiguous()
        y = harm_targets(harm)[ok]
        rms = float(torch.sqrt((y.double() ** 2).mean()).item())
        self.model.set_scales(1.0 / rms, self.err_calib)
        y = (y * self.out_scale).contiguous()
        mean = x.double().mean(0).cpu().numpy()
        std = x.double().std(0).cpu().numpy()
        std = np.where(std > 1e-6, std, 1.0)
        for net in self.nets:
            net.set_input_norm(mean, std)
        t0 = time.perf_counter()
        self._train(self.nets, x, [y, y], steps, batch, lr, lr_final, seed, log)
        if residual_steps > 0:
            if not self.model.residual:
                self.model.add_residual()
            res = []
            for net in self.nets:
                r = torch.empty_like(y)
                for b in range(0, x.shape[0], 1 << 16):
                    net.forward(x[b:b + (1 << 16)].contiguous(), out=r[b:b + (1 << 16)])
                res.append((y - r).contiguous())
            rrms = float(torch.sqrt(torch.stack([(r.double() ** 2).mean() for r in res]).mean()).item())
            self.model.set_residual_scale(1.0 / rrms)
            sc = np.float32(self.model.res_scale)
            for net in self.model.residual:
                net.set_input_norm(mean, std)
            self._train(self.model.residual, x, [(r * sc).contiguous() for r in res], residual_steps, batch, lr,
                        lr_final, seed + 1, log)
        torch.cuda.synchronize()
        self.train_seconds = time.perf_counter() - t0
        return self

    def _train(self, nets, x, targets, steps, batch, lr, lr_final, seed, log):
        torch = _torch()
        n = x.shape[0]
        g = torch.Generator(device=x.device)
        g.manual_seed(seed)
        for it in range(steps):
            lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
            for net, t in zip(nets, targets):
                idx = torch.randint(0, n, (min(batch, n),), device=x.device, generator=g)
                loss = net.train_step(x[idx].contiguous(), t[idx].contiguous(), lr_t)
            if log is not None and (it % max(steps // 10, 1) == 0 or it == steps - 1):
                log(f"step {it}: lr {lr_t:.2e} loss {float(loss.item()) / (min(batch, n) * t.shape[1]):.3e}")

    def raw(self, inst):
        """Per-member predictions (network units, the residual stage included) and the features' status."""
        x, st = self.ctx.surrogate_features(inst)
        out = [net.forward(x) for net in self.nets]
        if self.model.residual:
            inv = float(np.float32(1.0) / np.float32(self.model.res_scale))
            out = [o + net.forward(x) * inv for o, net in zip(out, self.model.residual)]
        return out, st

    def calibrate(self, inst, harm, quantile=0.99):
        """err_calib = quantile of (true relative L2 error) / (ensemble spread) over held-out instances,
        so that the estimate bounds the error of that fraction of them."""
        torch = _torch()
        (ya, yb), st = self.raw(inst)
        y = harm_targets(harm) * self.out_scale
        pred = 0.5 * (ya + yb)
        true = torch.linalg.vector_norm(pred - y, dim=1) / torch.linalg.vector_norm(y, dim=1)
        spread = 2.0 * torch.linalg.vector_norm(ya - yb, dim=1) / torch.linalg.vector_norm(ya + yb, dim=1)
        ok = (st == 0) & torch.isfinite(true) & torch.isfinite(spread) & (spread > 0)
        ratio = (true[ok] / spread[ok]).double().cpu().numpy()
        self.model.set_scales(self.out_scale, float(np.quantile(ratio, quantile)))
        return true[ok].double().cpu().numpy(), spread[ok].double().cpu().numpy()

    def predict(self, inst, L, drive, samples, settle, tol, substeps=0):
        """fpn_surrogate_predict: (harm, err_estimate, used_solver, status, n_fallback)."""
        return self.ctx.surrogate_predict(self.model, tol, inst, L, drive, samples, settle, self.n_harm,
                                          substeps=substeps)
