"""Training and evaluation of the learned velocity surrogate.

Orchestration only: features, labels, forward and backward passes and the
optimiser all run in librmdf kernels (``binding.mlp_*``); torch tensors are
the buffers.

* ``harvest``: run the search-mode filter (with feature output) over seeded
  flow scenes; collect, for sampled anchors of the last frame, the network
  input (1152 BF16 log-spectrum features), the search's velocity (label) and
  the scene's true background velocity.
* ``Trainer``: BF16 MFMA forward/backward, Adam on FP32 master weights.
* ``evaluate``: learned mode vs search mode on held-out seeds: velocity RMSE
  against the truth, prediction-error residual RMS away from the targets,
  fallback rate and pixel-frames/s.

Command line: ``python -m paper_1408_3526_amd.learned train --out PATH``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

N_IN, N_H1, N_H2, N_OUT = 1152, 128, 64, 3
M16 = (16, 16, 8)
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "velocity_mlp_16x16x8.npy")


def grid():
    from . import scenes
    return scenes.grid(-4, 4, 0.5)


def valid_mask(H, W, targets, t_out, dx=8, dy=8, radius=3.0, margin=15):
    """Anchors whose window is inside the frame and whose output pixel
    (anchor - m') is more than `radius` px from every target at frame t_out."""
    ys, xs = np.mgrid[0:H, 0:W]
    m = (xs >= margin) & (ys >= margin)
    px, py = xs - dx, ys - dy
    for tg in targets:
        cx, cy = tg[t_out]
        m &= (px - cx) ** 2 + (py - cy) ** 2 > radius * radius
    return m


def harvest(seeds, H=256, W=320, T=30, per_seq=40000, seed_sample=0, log=None):
    """Features (torch BF16 [N, 1152]), search labels and true velocities
    ([N, 2] float32) from the last frame of each seeded sequence."""
    import torch

    from . import binding, scenes
    g = grid()
    rng = np.random.default_rng(seed_sample)
    Xs, labs, trues = [], [], []
    for s in seeds:
        t0 = time.time()
        sc = scenes.flow_scene(int(s), H=H, W=W, T=T, n_targets=max(2, (H * W) // 16384),
                               band_width=(W / 16, W / 8))
        f = binding.Filter(H, W, *M16, g, g, write_features=True)
        dev = torch.from_numpy(sc.frames).cuda()
        for t in range(T):
            f.push_frame(dev[t])
        feats = f.features().reshape(H * W, N_IN)
        vxy, _ = f.velocity()
        torch.cuda.synchronize()
        f.close()
        mask = valid_mask(H, W, sc.targets, T - 1 - M16[2] // 2).reshape(-1)
        cand = np.flatnonzero(mask)
        sel = rng.choice(cand, size=min(per_seq, cand.size), replace=False)
        sel_t = torch.from_numpy(sel).cuda()
        Xs.append(feats.index_select(0, sel_t))
        labs.append(vxy.reshape(-1, 2).index_select(0, sel_t))
        # true background velocity at the output pixel (anchor - m')
        ys, xs = sel // W, sel % W
        trues.append(torch.from_numpy(sc.velocity[np.clip(ys - 8, 0, H - 1), np.clip(xs - 8, 0, W - 1)]
                                      .astype(np.float32)).cuda())
        if log:
            log("harvest seed %d: %d samples (%.1f s)" % (s, sel.size, time.time() - t0))
    return torch.cat(Xs), torch.cat(labs).contiguous(), torch.cat(trues).contiguous()


class Trainer:
    """FP32 master weights + Adam; BF16 copies feed the MFMA GEMMs."""

    def __init__(self, seed=0, lr=1e-3, wv=1.0, half_step=0.25, batch=4096):
        import torch
        self.torch = torch
        g = torch.Generator().manual_seed(seed)
        dev = "cuda"

        def he(o, i):
            return (torch.randn(o, i, generator=g) * np.sqrt(2.0 / i)).float().to(dev)

        self.p = {"W1": he(N_H1, N_IN), "b1": torch.zeros(N_H1, device=dev),
                  "W2": he(N_H2, N_H1), "b2": torch.zeros(N_H2, device=dev),
                  "W3": (torch.randn(N_OUT, N_H2, generator=g) * np.sqrt(1.0 / N_H2)).float().to(dev),
                  "b3": torch.zeros(N_OUT, device=dev)}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.bf = {"W1": torch.empty(N_H1, N_IN, dtype=torch.bfloat16, device=dev),
                   "W2": torch.empty(N_H2, N_H1, dtype=torch.bfloat16, device=dev)}
        from . import binding as b
        self.b = b
        b.mlp_to_bf16(self.p["W1"], self.bf["W1"])
        b.mlp_to_bf16(self.p["W2"], self.bf["W2"])
        self.lr, self.wv, self.half_step, self.batch = lr, wv, half_step, batch
        self.step_n = 0
        B = batch
        bf16 = torch.bfloat16
        self.buf = {"H1": torch.empty(B, N_H1, dtype=bf16, device=dev), "H2": torch.empty(B, N_H2, dtype=bf16, device=dev),
                    "dH2": torch.empty(B, N_H2, dtype=bf16, device=dev), "dH1": torch.empty(B, N_H1, dtype=bf16, device=dev),
                    "dH2t": torch.empty(N_H2, B, dtype=bf16, device=dev), "H1t": torch.empty(N_H1, B, dtype=bf16, device=dev),
                    "dH1t": torch.empty(N_H1, B, dtype=bf16, device=dev), "Xt": torch.empty(N_IN, B, dtype=bf16, device=dev),
                    "W2t": torch.empty(N_H1, N_H2, dtype=bf16, device=dev),
                    "loss": torch.zeros(1, device=dev)}

    def forward(self, X, H1, H2):
        b = self.b
        b.mlp_gemm_nt(X, self.bf["W1"], bias=self.p["b1"], epi=1, out_bf16=H1)
        b.mlp_gemm_nt(H1, self.bf["W2"], bias=self.p["b2"], epi=1, out_bf16=H2)

    def grads(self, X, lab):
        """Loss and gradients of one batch (into self.g); returns the loss tensor."""
        b, u = self.b, self.buf
        n = X.shape[0]
        H1, H2, dH2, dH1 = u["H1"][:n], u["H2"][:n], u["dH2"][:n], u["dH1"][:n]
        self.forward(X, H1, H2)
        for k in ("W3", "b3"):
            self.g[k].zero_()
        u["loss"].zero_()
        b.mlp_head(H2, self.p["W3"], self.p["b3"], lab, self.wv, self.half_step, dH2, self.g["W3"], self.g["b3"],
                   u["loss"])
        dH2t, H1t, dH1t, Xt = u["dH2t"][:, :n], u["H1t"][:, :n], u["dH1t"][:, :n], u["Xt"][:, :n]
        if n != self.batch:
            dH2t, H1t, dH1t, Xt = (self.torch.empty(t.shape[0], n, dtype=self.torch.bfloat16, device="cuda")
                                   for t in (dH2t, H1t, dH1t, Xt))
        b.mlp_transpose(dH2, dH2t)
        b.mlp_transpose(H1, H1t)
        b.mlp_gemm_nt(dH2t, H1t, out_f32=self.g["W2"])                         # dW2 = dH2^T H1
        b.mlp_colsum(dH2, self.g["b2"])
        b.mlp_transpose(self.bf["W2"], u["W2t"])
        b.mlp_gemm_nt(dH2, u["W2t"], epi=2, aux=H1, out_bf16=dH1)              # dH1 = dH2 W2 * (H1 > 0)
        b.mlp_transpose(dH1, dH1t)
        b.mlp_transpose(X, Xt)
        b.mlp_gemm_nt(dH1t, Xt, out_f32=self.g["W1"])                          # dW1 = dH1^T X
        b.mlp_colsum(dH1, self.g["b1"])
        return u["loss"]

    def step(self, X, lab):
        loss = self.grads(X, lab)
        self.step_n += 1
        for k in self.p:
            self.b.mlp_adam(self.p[k], self.g[k], self.m[k], self.v[k], self.bf.get(k), self.lr, self.step_n)
        return loss

    def blob(self):
        return np.concatenate([self.p[k].detach().cpu().numpy().ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def train(X, lab, steps=3000, batch=4096, lr=1e-3, seed=0, log=None):
    import torch
    tr = Trainer(seed=seed, lr=lr, batch=batch)
    N = X.shape[0]
    gen = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for s in range(steps):
        idx = torch.randint(0, N, (batch,), device="cuda", generator=gen)
        Xb = X.index_select(0, idx).contiguous()
        lb = lab.index_select(0, idx).contiguous()
        loss = tr.step(Xb, lb)
        if s % 200 == 0 or s == steps - 1:
            losses.append((s, float(loss.item())))
            if log:
                log("step %d loss %.4f" % losses[-1])
    return tr, losses


def residual_rms(out, targets, t_out, margin=15):
    H, W = out.shape
    m = valid_mask(H, W, targets, t_out, margin=margin)
    return float(np.sqrt(np.mean(out[m].astype(np.float64) ** 2)))


def evaluate(weights, seeds, H=512, W=640, T=40, thr=0.9, log=None):
    """Learned mode vs search mode on held-out seeds (same frames)."""
    import torch

    from . import binding, scenes
    g = grid()
    rows = []
    for s in seeds:
        sc = scenes.flow_scene(int(s), H=H, W=W, T=T, n_targets=20)
        dev = torch.from_numpy(sc.frames).cuda()
        res = {}
        for mode in ("search", "learned"):
            kw = dict(velocity_mode=binding.VEL_LEARNED, conf_threshold=thr) if mode == "learned" else {}
            f = binding.Filter(H, W, *M16, g, g, **kw)
            if mode == "learned":
                f.set_weights(weights)
            resid, rmse_v, fb = [], [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for t in range(T):
                f.push_frame(dev[t])
                if t >= T - 10:
                    out = f.output().cpu().numpy()
                    vxy, idx = f.velocity()
                    vxy, idx = vxy.cpu().numpy(), idx.cpu().numpy()
                    t_out = t - M16[2] // 2
                    resid.append(residual_rms(out, sc.targets, t_out))
                    m = valid_mask(H, W, sc.targets, t_out)
                    tv = sc.velocity[np.clip(np.arange(H) - 8, 0, H - 1)][:, np.clip(np.arange(W) - 8, 0, W - 1)]
                    rmse_v.append(float(np.sqrt(np.mean(np.sum((vxy[m] - tv[m]) ** 2, -1)))))
                    fb.append(float(np.mean(idx[m] >= 0)) if mode == "learned" else 1.0)
            torch.cuda.synchronize()
            f.close()
            res[mode] = {"residual_rms": float(np.mean(resid)), "velocity_rmse": float(np.mean(rmse_v)),
                         "fallback_rate": float(np.mean(fb))}
        rows.append(res)
        if log:
            log("eval seed %d: %s" % (s, json.dumps(res)))
    agg = {}
    for mode in ("search", "learned"):
        agg[mode] = {k: float(np.mean([r[mode][k] for r in rows])) for k in rows[0][mode]}
    return agg


def throughput(weights, H=512, W=640, T=24, steps=200, thr=0.9):
    """pixel-frames/s of search and learned mode on the same frames."""
    import torch

    from . import binding, scenes
    g = grid()
    sc = scenes.flow_scene(1, H=H, W=W, T=T, n_targets=20)
    dev = torch.from_numpy(sc.frames).cuda()
    out = {}
    for mode in ("search", "learned"):
        kw = dict(velocity_mode=binding.VEL_LEARNED, conf_threshold=thr) if mode == "learned" else {}
        f = binding.Filter(H, W, *M16, g, g, **kw)
        if mode == "learned":
            f.set_weights(weights)
        for t in range(T):
            f.push_frame(dev[t])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            f.push_frame(dev[i % T])
        e1.record()
        torch.cuda.synchronize()
        out[mode] = steps * H * W / (e0.elapsed_time(e1) / 1e3)
        f.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--train-seeds", type=int, default=50)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--per-seq", type=int, default=40000)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--report", default="")
    a = ap.parse_args(argv)

    def log(m):
        print(m, flush=True)

    rep = {}
    if a.cmd == "train":
        X, lab, true = harvest(range(1000, 1000 + a.train_seeds), per_seq=a.per_seq, log=log)
        log("dataset %s" % (tuple(X.shape),))
        tr, losses = train(X, lab, steps=a.steps, log=log)
        w = tr.blob()
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
        np.save(a.out, w.astype(np.float32))
        rep["train"] = {"samples": int(X.shape[0]), "steps": a.steps, "losses": losses}
        weights = w
    else:
        weights = np.load(a.weights)
    rep["eval"] = evaluate(weights, range(2000, 2000 + a.eval_seeds), log=log)
    rep["throughput"] = throughput(weights)
    log(json.dumps(rep))
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
