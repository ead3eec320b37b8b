"""Training and use of the learned surrogate of the exact orientation/size
average (SANS_MODE_SURROGATE).

Everything numerical runs in libsans kernels: targets (sans_pq_dataset, the
same Gauss-Legendre quadrature as SANS_MODE_QUAD), forward and backward
passes (BF16 MFMA GEMMs), the MSE gradient and Adam.  PyTorch holds the
device buffers and shuffles the dataset once per epoch.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import sans
from . import workloads as W

KIND = {"parallelepiped": sans.KIND["parallelepiped"], "spheroid": sans.KIND["ellipsoid"]}
DATA_KIND = {"parallelepiped": "parallelepiped", "spheroid": "ellipsoid"}

#: Where the trained networks are kept (BF16 weights, FP32 master copy and
#: the input box, safetensors).
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def weights_path(model: str) -> str:
    return os.path.join(WEIGHTS_DIR, f"surrogate_{model}.safetensors")


def normalise(x: np.ndarray | torch.Tensor, lo, hi):
    """u_k = (2 x_k - lo_k - hi_k)/(hi_k - lo_k) for the first 4 inputs (0
    where lo_k = hi_k); the other inputs stay 0."""
    u = x.clone() if isinstance(x, torch.Tensor) else x.copy()
    for k in range(4):
        if hi[k] > lo[k]:
            u[:, k] = (2 * x[:, k] - lo[k] - hi[k]) / (hi[k] - lo[k])
        else:
            u[:, k] = 0.0
    return u


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the flat parameter order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    fan = [8, 256, 256, 256]
    for l in range(4):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / fan[l]), size=fan[l] * 256))
        parts.append(np.zeros(256))
    parts.append(rng.normal(0.0, math.sqrt(1.0 / 256), size=256))
    parts.append(np.zeros(1))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == sans.sans_mlp_param_count()
    return w


def make_dataset(model: str, n: int, seed: int, quad_n: int = 76):
    """(u, t) on the device: normalised inputs and exact targets
    t = ln(<F^2>(q)/<F^2>(0)) - ln P_ref(q) (the network's residual)."""
    x = torch.from_numpy(W.surrogate_inputs(model, n, seed)).cuda()
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    chunk = 1 << 20
    for i in range(0, n, chunk):
        xi = x[i:i + chunk].contiguous()
        ti = torch.empty(xi.shape[0], dtype=torch.float32, device="cuda")
        sans.sans_pq_dataset(DATA_KIND[model], xi, ti, quad_n)
        t[i:i + chunk] = ti
    lo, hi = W.SURROGATE_BOX[model]
    return normalise(x, lo, hi).contiguous(), t


class Surrogate:
    """A network with FP32 master weights, its BF16 copy and Adam state."""

    def __init__(self, model: str, seed: int = 0):
        self.model = model
        self.lo, self.hi = W.SURROGATE_BOX[model]
        w = torch.from_numpy(init_params(seed)).cuda()
        self.w32 = w
        self.wb = torch.empty(w.numel(), dtype=torch.bfloat16, device="cuda")
        sans.sans_f32_to_bf16(self.w32, self.wb)
        self.m = torch.zeros_like(w)
        self.v = torch.zeros_like(w)
        self.dw = torch.zeros_like(w)
        self.step_count = 0
        self._ws = None
        self._ws_n = 0

    def _workspace(self, n: int):
        if self._ws is None or self._ws_n < n:
            nbytes = sans.sans_mlp_workspace_bytes(n)
            self._ws = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
            self._ws_n = n
        return self._ws

    def predict(self, u: torch.Tensor, batch: int = 1 << 16) -> torch.Tensor:
        out = torch.empty(u.shape[0], dtype=torch.float32, device="cuda")
        for i in range(0, u.shape[0], batch):
            ui = u[i:i + batch].contiguous()
            yi = torch.empty(ui.shape[0], dtype=torch.float32, device="cuda")
            sans.sans_mlp_forward(self.wb, ui, yi, self._workspace(ui.shape[0]))
            out[i:i + batch] = yi
        return out

    def train(self, u: torch.Tensor, t: torch.Tensor, steps: int, batch: int = 4096,
              lr: float = 2e-3, lr_min: float = 2e-5, seed: int = 0, log_every: int = 0,
              verbose: bool = False):
        """Adam with cosine learning-rate decay over `steps` minibatches; the
        dataset is reshuffled every epoch.  Returns the loss history (and
        prints each entry as it is taken when verbose)."""
        n = u.shape[0]
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        y = torch.empty(batch, dtype=torch.float32, device="cuda")
        dy = torch.empty(batch, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ws = self._workspace(batch)
        hist = []
        pos = n
        us = ts = None
        t0 = time.perf_counter()
        for k in range(steps):
            if pos + batch > n:
                perm = torch.randperm(n, device="cuda", generator=g)
                us, ts = u[perm].contiguous(), t[perm].contiguous()
                pos = 0
            ub, tb = us[pos:pos + batch], ts[pos:pos + batch]
            pos += batch
            sans.sans_mlp_forward(self.wb, ub, y, ws)
            sans.sans_mse_grad(y, tb, dy, loss)
            sans.sans_mlp_backward(self.wb, ub, dy, self.dw, ws)
            self.step_count += 1
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(steps, 1)))
            sans.sans_adam_step(self.w32, self.wb, self.dw, self.m, self.v, cur, self.step_count)
            if log_every and (k + 1) % log_every == 0:
                hist.append((k + 1, float(loss) / log_every, time.perf_counter() - t0))
                loss.zero_()
                if verbose:
                    print(f"step {hist[-1][0]:7d}  mse {hist[-1][1]:.3e}  {hist[-1][2]:7.1f} s", flush=True)
        torch.cuda.synchronize()
        return hist

    def attach(self, model_handle) -> None:
        sans.sans_model_attach_surrogate(model_handle, self.wb, self.lo, self.hi)

    def save(self, path: str, meta: dict | None = None) -> None:
        from safetensors.torch import save_file
        box = torch.tensor([self.lo, self.hi], dtype=torch.float64)
        md = {"model": self.model}
        if meta:
            md["train"] = json.dumps(meta)
        save_file({"w_bf16": self.wb.cpu(), "w_fp32": self.w32.cpu(), "box": box}, path, metadata=md)

    @classmethod
    def load(cls, model: str, path: str | None = None) -> "Surrogate":
        """A trained network (weights and input box) from its safetensors file."""
        from safetensors.torch import load_file
        t = load_file(path or weights_path(model))
        sg = cls(model)
        sg.w32.copy_(t["w_fp32"].cuda())
        sg.wb.copy_(t["w_bf16"].cuda())
        box = t["box"].numpy()
        sg.lo, sg.hi = tuple(float(v) for v in box[0]), tuple(float(v) for v in box[1])
        return sg

    def evaluate(self, u: torch.Tensor, t: torch.Tensor) -> dict:
        """Error of the network against targets ln P: on ln P and on P."""
        d = (self.predict(u) - t).double()
        rel = torch.expm1(d.abs())
        return {"n": int(u.shape[0]), "lnp_rms": float(d.pow(2).mean().sqrt()),
                "lnp_max": float(d.abs().max()), "p_rel_mean": float(rel.mean()),
                "p_rel_p99": float(torch.quantile(rel[:1 << 20].float(), 0.99)),
                "p_rel_max": float(rel.max())}


def main(argv=None):
    """Train one surrogate on the GPU (own kernels end to end) and write it."""
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--model", choices=sorted(KIND), required=True)
    ap.add_argument("--n", type=float, default=1e7, help="training samples")
    ap.add_argument("--n-val", type=float, default=2e5, help="held-out samples")
    ap.add_argument("--epochs", type=float, default=120)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    n, nv = int(a.n), int(a.n_val)
    t0 = time.perf_counter()
    u, t = make_dataset(a.model, n, seed=1000 + a.seed)
    uv, tv = make_dataset(a.model, nv, seed=2000 + a.seed)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    steps = int(a.epochs * n / a.batch)
    sg = Surrogate(a.model, seed=a.seed)
    t0 = time.perf_counter()
    print(f"training {a.model}: {n} samples, {steps} steps of {a.batch}", flush=True)
    sg.train(u, t, steps=steps, batch=a.batch, lr=a.lr, seed=a.seed,
             log_every=max(1, min(steps // 20, 5000)), verbose=True)
    t_train = time.perf_counter() - t0
    ev = sg.evaluate(uv, tv)
    meta = {"n": n, "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "seed": a.seed,
            "steps": steps, "dataset_s": round(t_data, 2), "train_s": round(t_train, 2),
            "validation": ev}
    out = a.out or weights_path(a.model)
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    sg.save(out, meta)
    print(json.dumps(dict(meta, model=a.model, out=out)), flush=True)


if __name__ == "__main__":
    main()
