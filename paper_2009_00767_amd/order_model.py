"""Learned expansion order per level: training data, training and the model file.

The order-prediction network (layout in include/fmm.h) is trained on
truncation errors that the method itself produces: for every system of a
training batch and every level k, the level's far field is evaluated at each
order p of the grid 4..24 with every other level held at the reference order
30, in FP64 on the GPU; the label is

    eps_k(p) = ||phi(p at level k, 30 elsewhere) - phi(30 everywhere)||_2
               / ||phi(30 everywhere)||_2        (norms over the system),

which is exactly level k's truncation error because the levels of the
shift-free method exchange no coefficients.  The network regresses
log10 eps_k(p) from three features of (system, level) -- k / 10,
log2(non-empty level-k boxes) / 20 and log10 ||q||_2 -- by full-batch Adam on
the GPU (fmm_mlp_train, the library's own forward and backward kernels).

``python -m paper_2009_00767_amd.order_model`` regenerates the packaged model
``order_model_log2d.json`` (needs a GPU).  Only the library and numpy are
used; nothing here computes potentials on the CPU.
"""
import json
import os
import sys

import numpy as np

from . import (FMM, FMM_FP64, FMM_LOG2D, FMM_MLP_NPARAM, FMM_NO_FIELD, fmm_mlp_adam_step,
               fmm_mlp_loss_grad, fmm_mlp_train)

P_GRID = np.arange(4, 25)
P_REF = 30
LABEL_FLOOR = 1e-16
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order_model_log2d.json")


def default_depth(n, lmax):
    """Tree depth used for a system of n particles when none is given (about 16
    per leaf), as in fmm_eval_batched."""
    if n <= 0:
        return 2
    return int(min(max(int(np.floor(np.log(n / 16.0) / np.log(4.0) + 0.5)), 2), lmax))


def features(pos, q, L, side=5.0, origin=(0.0, 0.0)):
    """Network inputs of levels 2..L of one system, [L - 1, 3] FP32 (the same
    quantities the library forms on the device)."""
    n = len(q)
    nl = 1 << L
    c = np.minimum(np.floor((pos - np.asarray(origin)) * (nl / side)).astype(np.int64), nl - 1)
    qn = np.float32(np.log10(max(float(np.sqrt(np.sum(q * q))), 1e-30)))
    out = np.zeros((max(L - 1, 0), 3), np.float32)
    for k in range(2, L + 1):
        sh = L - k
        boxes = np.unique(((c[:, 1] >> sh) << 20) | (c[:, 0] >> sh)).size if n else 0
        out[k - 2] = (k / 10.0, np.log2(max(boxes, 1)) / 20.0, qn)
    return out


def level_errors(systems, lmax):
    """Labels eps[s, k, i] (k = 2..lmax, order P_GRID[i]) for every system, from
    batched FP64 evaluations on the GPU; entries of levels deeper than a
    system's depth are NaN."""
    import torch
    off = np.zeros(len(systems) + 1, np.int64)
    off[1:] = np.cumsum([len(qs) for _, qs in systems])
    pos = torch.from_numpy(np.concatenate([ps for ps, _ in systems])).cuda()
    q = torch.from_numpy(np.concatenate([qs for _, qs in systems])).cuda()
    depths = np.array([default_depth(len(qs), lmax) for _, qs in systems], np.int32)
    f = FMM(FMM_LOG2D, levels=lmax, order=P_REF, precision=FMM_FP64, max_particles=int(off[-1]),
            max_systems=max(len(systems), 2), max_levels=lmax, flags=FMM_NO_FIELD)

    def run(orders):
        f.set_level_orders(orders)
        pot, _ = f.evaluate_batched(off, pos, q, sys_levels=depths)
        torch.cuda.synchronize()
        return pot.cpu().numpy()

    ref = run([0, 0] + [P_REF] * (lmax - 1))
    seg = [slice(off[s], off[s + 1]) for s in range(len(systems))]
    rnorm = np.array([np.linalg.norm(ref[sl]) for sl in seg])
    eps = np.full((len(systems), lmax + 1, len(P_GRID)), np.nan)
    for k in range(2, lmax + 1):
        for i, p in enumerate(P_GRID):
            orders = [0, 0] + [P_REF] * (lmax - 1)
            orders[k] = int(p)
            phi = run(orders)
            for s, sl in enumerate(seg):
                if depths[s] >= k and rnorm[s] > 0:
                    eps[s, k, i] = np.linalg.norm(phi[sl] - ref[sl]) / rnorm[s]
    f.close()
    return eps, depths


def training_set(systems, lmax):
    """(features [M, 3], log10 labels [M, 21]) over every (system, level)."""
    eps, depths = level_errors(systems, lmax)
    X, Y = [], []
    for s, (ps, qs) in enumerate(systems):
        L = int(depths[s])
        if L < 2 or len(qs) == 0:
            continue
        fe = features(ps, qs, L)
        for k in range(2, L + 1):
            X.append(fe[k - 2])
            Y.append(np.log10(np.maximum(eps[s, k], LABEL_FLOOR)))
    return np.asarray(X, np.float32), np.asarray(Y, np.float32)


def init_weights(seed, y_mean):
    """He-normal hidden weights, zero hidden biases, output bias = label mean."""
    rng = np.random.default_rng(seed)
    w = np.zeros(FMM_MLP_NPARAM, np.float32)
    o = 0
    for fan_out, fan_in in ((64, 3), (64, 64), (21, 64)):
        w[o:o + fan_out * fan_in] = rng.normal(0.0, np.sqrt(2.0 / fan_in), fan_out * fan_in)
        o += fan_out * fan_in
        if fan_out == 21:
            w[o:o + 21] = y_mean
        o += fan_out
    assert o == FMM_MLP_NPARAM
    return w


def train(X, Y, seed=0, schedule=((3000, 3e-3), (3000, 1e-3), (2000, 3e-4))):
    """Full-batch Adam on the GPU; returns (weights, loss history)."""
    import torch
    w = torch.from_numpy(init_weights(seed, Y.mean(axis=0))).cuda()
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    hist = []
    for steps, lr in schedule:
        hist.append(fmm_mlp_train(w, x, t, steps, lr))
    torch.cuda.synchronize()
    return w.cpu().numpy(), np.concatenate(hist)


def save_checkpoint(path, w, m1, m2, stage, step, losses):
    """Training state: weights, Adam's two moment estimates, the schedule stage
    and the step within it (Adam's bias correction counts from there), and the
    losses so far (host arrays; an .npz file written atomically)."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, w=np.asarray(w, np.float32), m1=np.asarray(m1, np.float32),
             m2=np.asarray(m2, np.float32), stage=np.int64(stage), step=np.int64(step),
             losses=np.asarray(losses, np.float32))
    os.replace(tmp, path)


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as d:
        st = {k: d[k] for k in ("w", "m1", "m2", "losses")}
        st["stage"], st["step"] = int(d["stage"]), int(d["step"])
    if st["w"].size != FMM_MLP_NPARAM or st["m1"].size != FMM_MLP_NPARAM:
        raise ValueError(f"{path}: not a checkpoint of the order network")
    return st


def train_resumable(X, Y, ckpt, seed=0, schedule=((3000, 3e-3), (3000, 1e-3), (2000, 3e-4)),
                    every=500, max_steps=None):
    """train() one Adam step at a time (the library's loss-gradient and Adam
    kernels), saving the whole state to `ckpt` every `every` steps and at the
    end, and resuming from `ckpt` when it exists.  Each schedule stage starts its
    moments at zero and its step count at one, as fmm_mlp_train does, so an
    uninterrupted run gives train()'s weights.  max_steps stops after that many
    steps of this call (an interruption, for tests).  Returns (weights,
    losses, finished)."""
    import torch
    if os.path.exists(ckpt):
        st = load_checkpoint(ckpt)
        w0, m10, m20 = st["w"], st["m1"], st["m2"]
        stage, step, losses = st["stage"], st["step"], list(st["losses"])
    else:
        w0 = init_weights(seed, Y.mean(axis=0))
        m10 = m20 = np.zeros(FMM_MLP_NPARAM, np.float32)
        stage, step, losses = 0, 0, []
    w = torch.from_numpy(np.array(w0, np.float32)).cuda()
    m1 = torch.from_numpy(np.array(m10, np.float32)).cuda()
    m2 = torch.from_numpy(np.array(m20, np.float32)).cuda()
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    grad = torch.empty_like(w)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    done = 0

    def snapshot():
        torch.cuda.synchronize()
        save_checkpoint(ckpt, w.cpu().numpy(), m1.cpu().numpy(), m2.cpu().numpy(), stage, step,
                        losses)

    while stage < len(schedule):
        steps, lr = schedule[stage]
        while step < steps:
            if max_steps is not None and done >= max_steps:
                snapshot()
                return w.cpu().numpy(), np.asarray(losses, np.float32), False
            fmm_mlp_loss_grad(w, x, t, grad, loss)
            losses.append(float(loss.item()))
            step += 1
            fmm_mlp_adam_step(w, grad, m1, m2, step, lr)
            done += 1
            if step % every == 0:
                snapshot()
        stage, step = stage + 1, 0
        m1.zero_()
        m2.zero_()
    snapshot()
    return w.cpu().numpy(), np.asarray(losses, np.float32), True


def save(weights, meta, path=MODEL_PATH):
    with open(path, "w") as fh:
        json.dump({"meta": meta, "weights": [float(v) for v in weights]}, fh)


def load(path=MODEL_PATH):
    with open(path) as fh:
        d = json.load(fh)
    w = np.asarray(d["weights"], np.float32)
    if w.size != FMM_MLP_NPARAM:
        raise ValueError(f"{path}: {w.size} parameters, expected {FMM_MLP_NPARAM}")
    return w, d.get("meta", {})


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    out = argv[0] if argv else MODEL_PATH
    import workloads
    lmax = 7
    systems = workloads.batched_systems(384, 2, seed=1005, nmin=512, nmax=131072)
    X, Y = training_set(systems, lmax)
    print(f"training samples: {len(X)}", flush=True)
    w, hist = train(X, Y, seed=7)
    print(f"loss: first {hist[0]:.4f} last {hist[-1]:.5f}", flush=True)
    meta = {
        "network": "3 -> 64 ReLU -> 64 ReLU -> 21, FP32",
        "training_set": "384 systems, N log-uniform in [512, 131072], uniform or Gaussian "
                        "mixture (workloads.batched_systems seed 1005), depths "
                        "clamp(round(log4(N/16)), 2, 7)",
        "labels": "log10 of level-k truncation error at p = 4..24 against p = 30, relative to "
                  "||phi||_2 per system, FP64 GPU evaluations, floor 1e-16",
        "samples": int(len(X)),
        "schedule": "full-batch Adam: 3000 steps lr 3e-3, 3000 lr 1e-3, 2000 lr 3e-4, seed 7",
        "final_loss": float(hist[-1]),
    }
    save(w, meta, out)
    print(f"wrote {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
