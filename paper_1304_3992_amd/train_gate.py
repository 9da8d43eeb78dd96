"""Trains the smoothing gate on the GPU with liblogfx's own forward, backward
and AdamW kernels.

    python -m paper_1304_3992_amd.train_gate --labels tests/golden/gate_labels.npz \
        tests/golden/gate_labels_2048.npz --out paper_1304_3992_amd/gate_weights.bin

The training tiles are the seeded 11-bit scenes of ``scenes.gate_tile``
(index i, noisy version); their labels (smooth or not) come from label
files, one per tile size: arrays ``label``, ``d_raw``, ``d_med`` (the
disagreement with the noise-free map without and with the hybrid median),
the tile ``size``, ``count`` and the generator's ``base_seed``.  The tiles
of each file are split in order: the first 80 % train, the next 10 %
validate (the epoch with the lowest validation loss is kept), the last 10 %
test.  Features are computed on the GPU by pass 1 (one batch call per chunk
of tiles) and stay resident in device memory for the whole run.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import logfx, scenes

def _noisy(job):
    _, i, size, base_seed, band = job
    return scenes.gate_tile(i, size, base_seed, twin=False, band=band)[0]


def _scene_tiles(job):
    seed, size, tile, locs = job
    base = scenes.config5_base(size, seed)
    return [scenes.config5_tile(base, b, ty, tx, tile, seed)[0] for b, ty, tx in locs]


def he_uniform(seed: int) -> np.ndarray:
    """Initial parameters (flat, FP32): He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in [(16, 3, 3, 3), (16,), (32, 16, 3, 3), (32,), (32, 32, 3, 3), (32,), (32,), (1,)]:
        if len(shape) > 1 or shape == (32,) and len(parts) == 6:
            fan_in = int(np.prod(shape[1:])) if len(shape) > 1 else shape[0]
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == logfx.GATE_NPARAM
    return theta


def default_params():
    t1, _ = logfx.make_log_mask(5, 0.8, 16)
    t2, _ = logfx.make_log_mask(9, 1.4, 16)
    return logfx.Params(t1, t2)


def compute_features(ctx, pool, jobs, log=print):
    """bfloat16 features [len(jobs), 3, 128, 128] of the noisy tiles, on the
    GPU.  A job is ("tile", index, size, base_seed, band) -- a
    scenes.gate_tile -- or ("scene", seed, scene_size, tile, band, ty, tx) --
    a tile of a four-band scene, scenes.config5_tile.  pool: worker
    processes that generate the tiles (started before the process touched
    the GPU)."""
    import torch
    n = len(jobs)
    feats = torch.empty((n, 3, logfx.GATE_CELLS, logfx.GATE_CELLS), dtype=torch.bfloat16, device="cuda")
    params = default_params()
    t0 = time.time()

    def run(rows, tiles):
        devs = [torch.from_numpy(t.view(np.int16)).cuda() for t in tiles]
        out = torch.empty((len(rows), 3, logfx.GATE_CELLS, logfx.GATE_CELLS), dtype=torch.bfloat16, device="cuda")
        ctx.gate_features(devs, params, out, bits=11)
        feats[torch.tensor(rows, device="cuda")] = out
        torch.cuda.synchronize()

    # tiles of scenes: one worker per scene builds the scene and cuts its tiles
    scene_rows = {}
    for r, j in enumerate(jobs):
        if j[0] == "scene":
            scene_rows.setdefault((j[1], j[2], j[3]), []).append(r)
    keys = list(scene_rows)
    for k0 in range(0, len(keys), 16):
        part = keys[k0:k0 + 16]
        got = pool.map(_scene_tiles, [(seed, size, tile, [jobs[r][4:7] for r in scene_rows[(seed, size, tile)]])
                                      for seed, size, tile in part])
        for key, tiles in zip(part, got):
            rows = scene_rows[key]
            for c0 in range(0, len(rows), 32):
                run(rows[c0:c0 + 32], tiles[c0:c0 + 32])
        log(f"features of {k0 + len(part)}/{len(keys)} scenes ({time.time() - t0:.0f} s)")
    # single tiles, about 256 Mpixel per chunk
    rows = [r for r, j in enumerate(jobs) if j[0] == "tile"]
    c0 = 0
    while c0 < len(rows):
        c1 = c0 + 1
        px = jobs[rows[c0]][2] ** 2
        while c1 < len(rows) and px + jobs[rows[c1]][2] ** 2 <= (1 << 28):
            px += jobs[rows[c1]][2] ** 2
            c1 += 1
        run(rows[c0:c1], pool.map(_noisy, [jobs[r] for r in rows[c0:c1]]))
        log(f"features {c1}/{len(rows)} ({time.time() - t0:.0f} s)")
        c0 = c1
    return feats


def evaluate(ctx, feats, labels_t, idx_np, batch):
    """(mean loss, logits numpy) over the samples idx_np."""
    import torch
    losses, logits = [], []
    for b0 in range(0, len(idx_np), batch):
        idx = torch.from_numpy(idx_np[b0:b0 + batch].astype(np.int32)).cuda()
        _, loss = ctx.gate_backward(feats, labels_t, idx, grad=False)
        z = ctx.gate_forward(feats, idx)
        losses.append(float(loss.cpu()[0]) * len(idx))
        logits.append(z.cpu().numpy())
    return sum(losses) / len(idx_np), np.concatenate(logits)


def gain_report(z, lab, d_raw, d_med):
    """Decision quality on a split, from the stored disagreements."""
    dec = z > 0
    d_gate = np.where(dec, d_med, d_raw)
    d_best = np.where(lab == 1, d_med, d_raw)
    return {"accuracy": float((dec == (lab == 1)).mean()), "smoothed_frac": float(dec.mean()),
            "D_never": float(d_raw.mean()), "D_always": float(d_med.mean()),
            "D_gated": float(d_gate.mean()), "D_best": float(d_best.mean())}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--labels", required=True, nargs="+", help="label files (one per tile size)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=0, help="tiles to use per file (0 = all)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--report", default="")
    a = ap.parse_args(argv)
    # the tile generators are forked before anything initialises the GPU
    pool = mp.get_context("fork").Pool(min(a.workers, 16))
    import torch
    if not torch.cuda.is_available():
        sys.exit("training runs on the GPU")
    jobs, labs, raws, meds, splits = [], [], [], [], []
    for path in a.labels:
        d = np.load(path)
        size = int(d["size"])
        count = min(a.count or int(d["count"]), int(d["count"]))
        o = len(jobs)
        if "scene_seed" in d:   # tiles of four-band scenes
            band = True
            jobs += [("scene", int(d["scene_seed"][i]), int(d["scene_size"]), int(d["tile"]), int(d["band"][i]),
                      int(d["ty"][i]), int(d["tx"][i])) for i in range(count)]
        else:
            seed = int(d["base_seed"]) if "base_seed" in d else 400000
            band = bool(int(d["band"])) if "band" in d else False
            jobs += [("tile", i, size, seed, band) for i in range(count)]
        labs.append(d["label"][:count].astype(np.float32))
        raws.append(d["d_raw"][:count].astype(np.float64))
        meds.append(d["d_med"][:count].astype(np.float64))
        n_tr, n_va = int(0.8 * count), int(0.1 * count)
        name = ("scenes" if "scene_seed" in d else f"size{size}") + ("b" if band and "scene_seed" not in d else "")
        splits.append((name, o + np.arange(n_tr), o + np.arange(n_tr, n_tr + n_va), o + np.arange(n_tr + n_va, count)))
    lab, d_raw, d_med = np.concatenate(labs), np.concatenate(raws), np.concatenate(meds)
    # every tile size weighs the same in an epoch: smaller training sets are
    # repeated up to the size of the largest
    n_max = max(len(sp[1]) for sp in splits)
    tr = np.concatenate([np.resize(sp[1], n_max) for sp in splits])
    va = np.concatenate([sp[2] for sp in splits])
    te = np.concatenate([sp[3] for sp in splits])
    log = lambda m: print(m, flush=True)  # noqa: E731

    with pool, logfx.Context(0) as ctx:
        feats = compute_features(ctx, pool, jobs, log=log)
        labels_t = torch.from_numpy(lab).cuda()
        ctx.gate_set_params(he_uniform(a.seed))
        rng = np.random.default_rng(a.seed)
        steps_per_epoch = max(1, len(tr) // a.batch)
        total = steps_per_epoch * a.epochs
        best = (float("inf"), None, -1)
        grad = torch.empty(logfx.GATE_NPARAM, dtype=torch.float32, device="cuda")
        step = 0
        t0 = time.time()
        for ep in range(a.epochs):
            perm = rng.permutation(tr)
            tl = []
            for s in range(steps_per_epoch):
                idx = torch.from_numpy(perm[s * a.batch:(s + 1) * a.batch].astype(np.int32)).cuda()
                lr = a.lr * 0.5 * (1 + np.cos(np.pi * step / total))   # cosine decay
                _, loss = ctx.gate_backward(feats, labels_t, idx, grad=grad)
                ctx.gate_step(lr, grad)
                tl.append(loss)
                step += 1
            train_loss = float(torch.cat(tl).mean().cpu())
            vl, zv = evaluate(ctx, feats, labels_t, va, a.batch)
            acc = float(((zv > 0) == (lab[va] == 1)).mean())
            log(f"epoch {ep + 1}/{a.epochs}: train loss {train_loss:.4f}, val loss {vl:.4f}, "
                f"val acc {acc:.4f} ({time.time() - t0:.1f} s)")
            if vl < best[0]:
                best = (vl, ctx.gate_get_params(), ep + 1)
        ctx.gate_set_params(best[1])
        ctx.gate_save(a.out)
        rep = {"best_epoch": best[2], "val_loss": best[0], "train_seconds": time.time() - t0,
               "tiles": len(jobs)}
        for name, _, sva, ste in splits:
            _, zt = evaluate(ctx, feats, labels_t, ste, a.batch)
            _, zv = evaluate(ctx, feats, labels_t, sva, a.batch)
            rep[name] = {"val": gain_report(zv, lab[sva], d_raw[sva], d_med[sva]),
                                  "test": gain_report(zt, lab[ste], d_raw[ste], d_med[ste])}
        log(json.dumps(rep))
        if a.report:
            with open(a.report, "w") as f:
                json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
