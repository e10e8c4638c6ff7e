"""Learned acceptance / order selector: training data, GPU training, model files.

Every numerical step runs in the library's kernels: the candidate export and the labels
(``fmm_mac_training_data``), the forward/backward passes (``fmm_mlp_grad``,
``fmm_mlp_forward``) and the optimiser (``fmm_mlp_adam``).  This module orchestrates
them; torch tensors only hold device memory.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import struct

import numpy as np

from . import FMMError, Params, Tree, _check, _dev64, _stream, lib

NFEAT, NHID, NCLS, NPARAM = 16, 64, 8, 5768
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "mac_clustered.bin")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def reference_forces(tree: Tree, prm: Params):
    """Total short-range acceleration used to scale the label errors: the library's plain
    FP64 evaluation at order 8 and theta 0.3 (well below the bar)."""
    ref = Params.from_buffer_copy(prm)
    ref.p, ref.theta, ref.precision, ref.learned = 8, 0.3, 0, 0
    return tree.short_range(ref)


def training_data(pos, mass, prm: Params, theta_max=0.55, eps=5e-5, stride=1, cap=4_000_000, with_pairs=False):
    """Candidate pairs of a box with their features, labels (class 0 open, c = order - 1)
    and per-order measured errors."""
    import torch
    tree = Tree().build(pos, mass, prm)
    aref = reference_forces(tree, prm)
    dev = pos.device
    feats = torch.empty((cap, NFEAT), dtype=torch.float32, device=dev)
    labels = torch.empty(cap, dtype=torch.int32, device=dev)
    errs = torch.empty((cap, 7), dtype=torch.float32, device=dev)
    pairs = torch.empty((cap, 3), dtype=torch.int64, device=dev) if with_pairs else None
    cnt = C.c_int64()
    _check(lib().fmm_mac_training_data(tree._h, C.byref(prm), float(theta_max), _dev64(aref), float(eps), int(stride),
                                       _ptr(feats), _ptr(labels), _ptr(errs), _ptr(pairs), int(cap), C.byref(cnt),
                                       _stream(None)))
    n = cnt.value
    out = dict(feats=feats[:n].clone(), labels=labels[:n].clone(), errs=errs[:n].clone(), aref=aref)
    if with_pairs:
        out["pairs"] = pairs[:n].clone()
    tree.free()
    return out


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    w = np.zeros(NPARAM, np.float32)
    w[0:1024] = rng.standard_normal(1024) * np.sqrt(2.0 / NFEAT)
    w[1088:5184] = rng.standard_normal(4096) * np.sqrt(2.0 / NHID)
    w[5248:5760] = rng.standard_normal(512) * np.sqrt(1.0 / NHID)
    return w


def grad(params, mu, isd, X, y, class_w):
    """Loss and gradient on the device (fmm_mlp_grad)."""
    import torch
    g = torch.empty(NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().fmm_mlp_grad(_ptr(params), _ptr(mu), _ptr(isd), _ptr(X), _ptr(y), _ptr(class_w), int(X.shape[0]),
                              _ptr(g), _ptr(loss), _stream(None)))
    return float(loss.item()), g


def grad_noalloc(params, mu, isd, X, y, class_w, g, loss):
    """fmm_mlp_grad_noalloc: loss and gradient into the caller's g (5768 floats) and loss
    (1 float) with the library's fixed scratch (B <= 8192); allocates nothing."""
    _check(lib().fmm_mlp_grad_noalloc(_ptr(params), _ptr(mu), _ptr(isd), _ptr(X), _ptr(y), _ptr(class_w),
                                      int(X.shape[0]), _ptr(g), _ptr(loss), _stream(None)))


def forward(params, mu, isd, X):
    import torch
    Z = torch.empty((X.shape[0], NCLS), dtype=torch.float32, device=X.device)
    _check(lib().fmm_mlp_forward(_ptr(params), _ptr(mu), _ptr(isd), _ptr(X), int(X.shape[0]), _ptr(Z),
                                 _stream(None)))
    return Z


def adam(params, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    _check(lib().fmm_mlp_adam(_ptr(params), _ptr(g), _ptr(m), _ptr(v), int(step), float(lr), float(b1), float(b2),
                              float(eps), float(wd), _stream(None)))


def decode(logits_np, safety):
    c = logits_np.argmax(1)
    return np.where(c == 0, 0, np.minimum(c + 1 + safety, 8))


def needed_order(labels_np):
    return np.where(labels_np == 0, 99, labels_np + 1)  # 99: the pair must be opened


def unsafe_fraction(pred_order, labels_np):
    need = needed_order(labels_np)
    acc = pred_order >= 2
    return float(np.mean(acc & (pred_order < need)))


def train(feats, labels, epochs=40, batch=8192, lr=2e-3, wd=1e-5, seed=0, val_frac=0.1, log=None):
    """Train on the device with Adam; returns the model dict (numpy arrays) and history."""
    import torch
    dev = feats.device
    n = feats.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = max(1, int(val_frac * n))
    val_idx = torch.as_tensor(perm[:nval], device=dev)
    tr_idx = perm[nval:]
    Xtr_all = feats.index_select(0, torch.as_tensor(tr_idx, device=dev))
    x_np = Xtr_all.cpu().numpy().astype(np.float64)
    mu_np = x_np.mean(0).astype(np.float32)
    sd = x_np.std(0)
    isd_np = (1.0 / np.where(sd > 1e-6, sd, 1.0)).astype(np.float32)
    lab_np = labels.cpu().numpy()
    freq = np.bincount(lab_np[tr_idx], minlength=NCLS).astype(np.float64) + 1.0
    cw_np = (freq.sum() / freq) ** 0.5
    cw_np = (cw_np / cw_np.mean()).astype(np.float32)
    mu = torch.as_tensor(mu_np, device=dev)
    isd = torch.as_tensor(isd_np, device=dev)
    cw = torch.as_tensor(cw_np, device=dev)
    w = torch.as_tensor(init_params(seed), device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    step = 0
    hist = []
    Xval, yval = feats.index_select(0, val_idx), labels.index_select(0, val_idx)
    for ep in range(epochs):
        order = rng.permutation(len(tr_idx))
        tot = 0.0
        nb = 0
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))
        for b0 in range(0, len(order), batch):
            sel = torch.as_tensor(tr_idx[order[b0:b0 + batch]], device=dev)
            if sel.numel() < 32:
                continue
            X = feats.index_select(0, sel).contiguous()
            y = labels.index_select(0, sel).contiguous()
            loss, g = grad(w, mu, isd, X, y, cw)
            step += 1
            adam(w, g, m, v, step, lr_ep, wd=wd)
            tot += loss
            nb += 1
        Z = forward(w, mu, isd, Xval.contiguous()).cpu().numpy()
        yv = yval.cpu().numpy()
        accv = float(np.mean(Z.argmax(1) == yv))
        hist.append(dict(epoch=ep, loss=tot / max(nb, 1), val_acc=accv,
                         unsafe0=unsafe_fraction(decode(Z, 0), yv), unsafe1=unsafe_fraction(decode(Z, 1), yv)))
        if log:
            log(hist[-1])
    return dict(params=w.cpu().numpy(), mu=mu_np, isd=isd_np, adam_m=m.cpu().numpy(), adam_v=v.cpu().numpy(),
                step=step, class_w=cw_np, history=hist, val_logits=Z, val_labels=yv)


def select_safety(pos, mass, prm: Params, params, mu, isd, theta_max, target=5e-4, max_safety=6):
    """Smallest safety margin whose forces on a held-out box stay within `target` of the
    library's own FP64 reference (order 8, theta 0.3) at the 99th percentile, with the
    per-margin p99 values.  `prm` carries the box's split parameters and FP32/FP64 form."""
    import torch
    tree = Tree().build(pos, mass, prm)
    ref = reference_forces(tree, prm)
    rn = ref.norm(dim=1)
    floor = rn[rn > 0].median()
    run = Params.from_buffer_copy(prm)
    run.learned = 1
    p99 = {}
    chosen = max_safety
    try:
        for sf in range(max_safety + 1):
            set_model(params, mu, isd, theta_max, sf)
            got = tree.short_range(run)
            e = (got - ref).norm(dim=1) / torch.where(rn > 0, rn, floor)
            p99[sf] = float(torch.quantile(e, 0.99).item())
            if p99[sf] <= target:
                chosen = sf
                break
    finally:
        tree.free()
    return chosen, p99


def save_model(path, model, theta_max, eps, safety, config):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    cfg = json.dumps(config, sort_keys=True).encode()
    with open(path, "wb") as f:
        f.write(b"HFMMMAC1")
        f.write(struct.pack("<4i", 1, NFEAT, NHID, NCLS))
        f.write(struct.pack("<2d", float(theta_max), float(eps)))
        f.write(struct.pack("<2i", int(safety), 0))
        for a in (model["mu"], model["isd"], model["params"], model["adam_m"], model["adam_v"]):
            f.write(np.ascontiguousarray(a, np.float32).tobytes())
        f.write(struct.pack("<q", int(model["step"])))
        f.write(struct.pack("<i", len(cfg)))
        f.write(cfg)


def read_model(path):
    with open(path, "rb") as f:
        if f.read(8) != b"HFMMMAC1":
            raise FMMError(-1, "not a selector model file")
        ver, nf, nh, nc = struct.unpack("<4i", f.read(16))
        theta_max, eps = struct.unpack("<2d", f.read(16))
        safety, _ = struct.unpack("<2i", f.read(8))
        mu = np.frombuffer(f.read(4 * NFEAT), np.float32)
        isd = np.frombuffer(f.read(4 * NFEAT), np.float32)
        params = np.frombuffer(f.read(4 * NPARAM), np.float32)
        m = np.frombuffer(f.read(4 * NPARAM), np.float32)
        v = np.frombuffer(f.read(4 * NPARAM), np.float32)
        step, = struct.unpack("<q", f.read(8))
        ln, = struct.unpack("<i", f.read(4))
        cfg = json.loads(f.read(ln).decode())
    return dict(theta_max=theta_max, eps=eps, safety=safety, mu=mu, isd=isd, params=params, adam_m=m, adam_v=v,
                step=step, config=cfg)


def load_model(path=DEFAULT_MODEL):
    _check(lib().fmm_load_mac_model(str(path).encode()))


def set_model(params, mu, isd, theta_max, safety):
    p = np.ascontiguousarray(params, np.float32)
    mu = np.ascontiguousarray(mu, np.float32)
    isd = np.ascontiguousarray(isd, np.float32)
    _check(lib().fmm_set_mac_model(p.ctypes.data, mu.ctypes.data, isd.ctypes.data, float(theta_max), int(safety)))


def unload_model():
    _check(lib().fmm_set_mac_model(None, None, None, 0.0, 0))


def infer(X):
    """Logits of the loaded model through the BF16 MFMA path of the traversal."""
    import torch
    Z = torch.empty((X.shape[0], NCLS), dtype=torch.float32, device=X.device)
    _check(lib().fmm_mlp_infer(_ptr(X), int(X.shape[0]), _ptr(Z), _stream(None)))
    return Z
