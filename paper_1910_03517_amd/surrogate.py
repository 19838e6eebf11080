"""The learned surrogate of the estimate: weights, workspace, dataset,
training and inference, driving the library's kernels.

A small MLP (576 -> 256 -> 256 -> 6, ReLU) maps the normalised 64-bin
histograms of a (camera, side, block) unit's whole frame, own band and
facing band to the unit's affine maps; it is trained in float32 on the
plain estimator's output by the library's forward, backward and Adam
kernels.  At inference the plain estimate is always computed too: it judges
the network, and replaces its output wherever the residual exceeds `tol` or
an output is not finite.  The feature, residual and fallback definitions are
those of include/ringcorr.h.

This module allocates device buffers and sequences library calls; every
computation runs in the library's kernels.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

from . import rt, synth


class Workspace:
    """Device buffers of one surrogate estimate for a context with U = K*2*NB units."""

    def __init__(self, sizes: rt.rt_sizes, device="cuda"):
        import torch
        K, NB = sizes.n_cams, sizes.n_blocks
        U = K * 2 * NB
        e = dict(device=device)
        self.n = U
        self.X = torch.zeros((U, rt.MLP_IN), dtype=torch.float32, **e)
        self.H1 = torch.zeros((U, rt.MLP_HID), dtype=torch.float32, **e)
        self.H2 = torch.zeros((U, rt.MLP_HID), dtype=torch.float32, **e)
        self.Y = torch.zeros((U, rt.MLP_OUT), dtype=torch.float32, **e)
        self.T = torch.zeros((U, rt.MLP_OUT), dtype=torch.float32, **e)
        self.mask = torch.zeros(U, dtype=torch.uint8, **e)
        self.p_new = torch.zeros((K, 2, NB, rt.CSLOTS, 2), dtype=torch.float64, **e)
        self.status = torch.zeros((K, 2, NB, rt.CSLOTS), dtype=torch.int32, **e)
        self.used = torch.zeros(U, dtype=torch.uint8, **e)
        self.residual = torch.zeros(U, dtype=torch.float32, **e)


class Surrogate:
    """Inference with fallback, on one context."""

    def __init__(self, weights: rt.MlpTensors, tol: float = 1e-3):
        self.w = weights
        self.tol = tol

    def estimate(self, rig: rt.Rig, whole_hist_prev, ws: Workspace, stream=None) -> None:
        """Replace rt_estimate: features, plain estimate, network, choice, state update.
        The band statistics of the frame-set must be in rig.bufs."""
        b, ctx = rig.bufs, rig.ctx
        rt.rt_surrogate_features(ctx, b.band_hist, whole_hist_prev, ws.X, stream)
        rt.rt_estimate_new(ctx, b.band_sums, ws.p_new, ws.status, stream)
        rt.rt_mlp_forward(self.w, ws.X, ws.n, ws.H1, ws.H2, ws.Y, stream)
        rt.rt_surrogate_select(ctx, ws.Y, ws.p_new, ws.status, self.tol, b.params, b.valid, ws.used, ws.residual,
                               stream)

    def frameset(self, rig: rt.Rig, frames, out_frames, whole_hist_prev, ws: Workspace, stream=None) -> None:
        """One frame-set with the surrogate estimate (rt_surrogate_frameset);
        the whole-frame statistics of this frame-set land in rig.bufs (the next
        call's whole_hist_prev)."""
        rt.rt_surrogate_frameset(rig.ctx, self.w, self.tol, frames, out_frames, rig.bufs, whole_hist_prev, ws, stream)

    def frameset_stepwise(self, rig: rt.Rig, frames, out_frames, whole_hist_prev, ws: Workspace,
                          stream=None) -> None:
        """The same frame-set as the sequence of the fine-grained calls."""
        b = rig.bufs
        rt.rt_stats(rig.ctx, frames, b.band_hist, b.band_sums, None, None, stream)
        self.estimate(rig, whole_hist_prev, ws, stream)
        rt.rt_build_lut(rig.ctx, b.params, b.valid, b.lut8, b.q16, b.weights, stream)
        rt.rt_apply(rig.ctx, frames, out_frames, b.lut8, b.q16, b.weights, b.whole_hist, b.whole_sums, stream)


# ----------------------------------------------------------------------------- dataset

@dataclass
class Dataset:
    X: object            # torch float32 [N][576] on the device
    T: object            # torch float32 [N][6]
    rig_of_row: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))


def rig_specs(kind: str):
    """Camera rings the dataset is drawn from."""
    if kind == "rig14":
        return [synth.CamSpec(1920, 1080, 3, 8, 0, p) for p in range(14)]
    if kind == "small":
        return [synth.CamSpec(480, 272, 3, 8, 0, p) for p in range(6)]
    raise ValueError(kind)


def build_dataset(kind: str, n_bases: int, draws_per_base: int, seed: int, opts: rt.Options = rt.Options(),
                  device="cuda") -> Dataset:
    """Units of seeded synthetic rigs with fresh gains: features (whole-frame
    histogram of the same frame-set) and targets from the plain estimator,
    keeping the units whose three channels hold an estimate."""
    import torch
    specs = rig_specs(kind)
    cams = [rt.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos).with_pitch() for c in specs]
    rig = rt.Rig(cams, opts)
    ws = Workspace(rig.sizes, device)
    dist = rig.alloc_frames()
    b = rig.bufs
    Xs, Ts, owner = [], [], []
    for base_i in range(n_bases):
        spec = synth.RigSpec(f"dataset {kind}", 1000 + seed, specs)
        base = rig.upload(synth.rig_frames(spec, 0, seed=1000 * seed + base_i, distortion=False))
        grng = np.random.default_rng([1910, 31, seed, base_i])
        for d in range(draws_per_base):
            gains = synth.draw_gains(len(cams), 3, grng)
            synth.distort_device(base, gains, cams, dist)
            rt.rt_stats(rig.ctx, dist, b.band_hist, b.band_sums, b.whole_hist, b.whole_sums)
            rt.rt_surrogate_features(rig.ctx, b.band_hist, b.whole_hist, ws.X)
            rt.rt_estimate_new(rig.ctx, b.band_sums, ws.p_new, ws.status)
            rt.rt_surrogate_targets(rig.ctx, ws.p_new, ws.status, ws.T, ws.mask)
            keep = ws.mask.bool()
            Xs.append(ws.X[keep].clone())
            Ts.append(ws.T[keep].clone())
            owner.append(np.full(int(keep.sum().item()), base_i * draws_per_base + d, np.int32))
    torch.cuda.synchronize()
    rig.close()
    return Dataset(torch.cat(Xs), torch.cat(Ts), np.concatenate(owner))


# ----------------------------------------------------------------------------- training

class Trainer:
    """Mini-batch Adam on the mean squared error, all in the library's kernels."""

    def __init__(self, init: dict, lr: float = 1e-3, batch: int = 1024, seed: int = 0, device="cuda"):
        import torch
        self.w = rt.MlpTensors(init, device)
        self.g = rt.MlpTensors(None, device)
        self.m = rt.MlpTensors(None, device)
        self.v = rt.MlpTensors(None, device)
        self.lr, self.batch, self.step = lr, batch, 0
        self.rng = np.random.default_rng([1910, 41, seed])
        e = dict(device=device, dtype=torch.float32)
        B = batch
        self.xb = torch.zeros((B, rt.MLP_IN), **e)
        self.tb = torch.zeros((B, rt.MLP_OUT), **e)
        self.h1 = torch.zeros((B, rt.MLP_HID), **e)
        self.h2 = torch.zeros((B, rt.MLP_HID), **e)
        self.y = torch.zeros((B, rt.MLP_OUT), **e)
        self.dy = torch.zeros((B, rt.MLP_OUT), **e)
        self.dz1 = torch.zeros((B, rt.MLP_HID), **e)
        self.dz2 = torch.zeros((B, rt.MLP_HID), **e)
        self.loss = torch.zeros(1, **e)
        self.device = device

    def epoch(self, data: Dataset) -> float:
        """One pass over a seeded permutation of the dataset (whole mini-batches),
        enqueued by the library in one call; returns the mean batch loss."""
        import torch
        n = data.X.shape[0]
        steps = n // self.batch
        perm = torch.as_tensor(self.rng.permutation(n).astype(np.int32), device=self.device)
        if steps == 0:
            return float("nan")
        losses = torch.zeros(steps, dtype=torch.float32, device=self.device)
        work = {"xb": self.xb, "tb": self.tb, "h1": self.h1, "h2": self.h2, "y": self.y, "dy": self.dy,
                "dz1": self.dz1, "dz2": self.dz2}
        rt.rt_mlp_train(self.w, self.g, self.m, self.v, data.X, data.T, perm, self.batch, steps, self.step + 1,
                        self.lr, work, losses)
        self.step += steps
        return float(losses.mean().item())

    def epoch_stepwise(self, data: Dataset) -> float:
        """The same epoch as separate library calls per step (the reference for epoch)."""
        import torch
        n = data.X.shape[0]
        perm = torch.as_tensor(self.rng.permutation(n).astype(np.int32), device=self.device)
        losses = []
        for s in range(0, n - self.batch + 1, self.batch):
            idx = perm[s:s + self.batch]
            B = self.batch
            rt.rt_gather_rows(data.X, rt.MLP_IN, idx, B, self.xb)
            rt.rt_gather_rows(data.T, rt.MLP_OUT, idx, B, self.tb)
            rt.rt_mlp_forward(self.w, self.xb, B, self.h1, self.h2, self.y)
            rt.rt_mlp_backward(self.w, self.xb, self.h1, self.h2, self.y, self.tb, B, self.g, self.dy, self.dz1,
                               self.dz2)
            self.step += 1
            rt.rt_mlp_adam(self.w, self.g, self.m, self.v, self.step, self.lr)
            rt.rt_mlp_mse(self.y, self.tb, B, self.loss)
            losses.append(self.loss.clone())
        return float(torch.stack(losses).mean().item()) if losses else float("nan")

    def save(self, path: str) -> None:
        """Checkpoint: weights, Adam moments, step count, learning rate, batch
        size and the state of the mini-batch permutation generator, so that
        training resumed from it continues bit for bit as it would have."""
        arr = {}
        for tag, t in (("w", self.w), ("m", self.m), ("v", self.v)):
            for k, v in t.host().items():
                arr[f"{tag}_{k}"] = v
        arr["step"] = np.array(self.step, np.int64)
        arr["lr"] = np.array(self.lr, np.float64)
        arr["batch"] = np.array(self.batch, np.int64)
        arr["rng_state"] = np.array(json.dumps(self.rng.bit_generator.state))
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        np.savez(path, **arr)

    def load(self, path: str) -> None:
        """Restore a checkpoint written by save (plain arrays and a JSON
        string; nothing in the file is executed)."""
        import torch
        with np.load(path, allow_pickle=False) as z:
            if int(z["batch"]) != self.batch:
                raise ValueError(f"checkpoint batch {int(z['batch'])} differs from the trainer's {self.batch}")
            for tag, t in (("w", self.w), ("m", self.m), ("v", self.v)):
                for k in rt.MlpTensors.NAMES:
                    getattr(t, k).copy_(torch.as_tensor(z[f"{tag}_{k}"], device=self.device))
            self.step = int(z["step"])
            self.lr = float(z["lr"])
            state = json.loads(str(z["rng_state"]))
        rng = np.random.default_rng()
        rng.bit_generator.state = state
        self.rng = rng


def predict(w: rt.MlpTensors, X, device="cuda"):
    """Network outputs for rows X (device float32 [N][576])."""
    import torch
    n = X.shape[0]
    e = dict(device=device, dtype=torch.float32)
    h1, h2 = torch.zeros((n, rt.MLP_HID), **e), torch.zeros((n, rt.MLP_HID), **e)
    y = torch.zeros((n, rt.MLP_OUT), **e)
    rt.rt_mlp_forward(w, X, n, h1, h2, y)
    return y

