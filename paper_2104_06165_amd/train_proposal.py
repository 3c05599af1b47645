"""Train the learned initial-plane proposal network on the GPU.

Teacher: the plain PatchMatch depth-map estimation (random initialisation, 8 red/black
iterations) of this library on seeded synthetic 1600x1066 scenes (the high-resolution
scene recipe: 25 planes, 35% texture-less, depth 1-20 m, 10 sources; 21x21 window at
dilation 2, top-5).  Each scene gives one training sample at 1/4 resolution: the network
input of the reference view and the teacher's planes as targets, masked to blocks whose
teacher cost is below ``--max-cost``.

Samples are produced and consumed on the GPU: a scene is rendered, the teacher runs, the
sample joins a device-resident buffer, and ``--steps-per-scene`` Adam steps on random
minibatches of the buffer follow.  After the last scene, ``--final-steps`` more steps run
over the whole buffer.  Every kernel (teacher, input builder, targets, forward, backward,
Adam) is the library's; torch only holds the buffers.

The run can be split: ``--init`` continues from a saved parameter vector, ``--seeds``
selects a slice of the training seeds.  The output is a float32 ``.npy`` parameter vector
(layout of include/phimvs_net.h) and a JSON log next to it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SHAPES = ((5, 32), (32, 32), (32, 32), (32, 32), (32, 4))


def initial_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases except the normal outputs (0, 0, -1): a fronto-parallel
    plane facing the camera at mid depth before any training."""
    r = np.random.default_rng(seed)
    out = []
    for l, (ci, co) in enumerate(SHAPES):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if l == len(SHAPES) - 1 else 1.0)
        w = r.normal(0.0, std, (9, ci, co))
        b = np.zeros(co)
        if l == len(SHAPES) - 1:
            b[3] = -1.0
        out.append(np.concatenate([w.ravel(), b]))
    return np.concatenate(out).astype(np.float32)


def log(*a):
    print(*a, flush=True)


def main(argv=None):
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--seeds", default="0:2000", help="slice a:b of the training seeds 100000..101999")
    ap.add_argument("--init", default=None, help="start from this .npy parameter vector")
    ap.add_argument("--out", required=True, help="output .npy parameter vector")
    ap.add_argument("--steps-per-scene", type=int, default=6)
    ap.add_argument("--final-steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=2e-4, help="learning rate of the final steps")
    ap.add_argument("--normal-weight", type=float, default=1.0)
    ap.add_argument("--max-cost", type=float, default=0.5, help="teacher cost threshold of the mask")
    ap.add_argument("--time-limit", type=float, default=1e9, help="stop adding scenes after this many seconds")
    ap.add_argument("--seed", type=int, default=7, help="initialisation and minibatch seed")
    args = ap.parse_args(argv)

    a, b = (int(v) for v in args.seeds.split(":"))
    seeds = list(sg.PROPOSAL_TRAIN_SEEDS)[a:b]
    cfg = sg.CONFIGS["proposal_train"]
    sol = sg.SOLVER["proposal_train"]
    W, H = cfg.width, cfg.height
    h, w = (H + 3) // 4, (W + 3) // 4
    dev = torch.device("cuda", 0)

    ctx = pm.Context(0)
    net = pm.Net(0)
    params = np.load(args.init) if args.init else initial_params(args.seed)
    net.set_params(params)
    rng = np.random.default_rng(args.seed + a)

    cap = len(seeds)
    X = torch.empty((cap, h, w, 5), dtype=torch.float32, device=dev)
    T = torch.empty((cap, h, w, 4), dtype=torch.float32, device=dev)
    M = torch.empty((cap, h, w), dtype=torch.float32, device=dev)
    D = torch.empty((cap, 2), dtype=torch.float32, device=dev)
    n = 0
    history = []
    t0 = time.time()
    solver_params = pm.Params(top_k=sol["top_k"], sigma_spatial_px=(sol["window"] - 1) / 2.0, seed=sg.PM_SEED)

    def train_steps(k, lr):
        losses = []
        for _ in range(k):
            idx = torch.from_numpy(rng.integers(0, n, min(args.batch, n))).to(dev)
            loss, _ = net.loss_grad(X[idx].contiguous(), T[idx].contiguous(), M[idx].contiguous(),
                                    D[idx].contiguous(), args.normal_weight, want_loss=True)
            net.adam(lr)
            losses.append(loss)
        return losses

    for i, s in enumerate(seeds):
        if time.time() - t0 > args.time_limit:
            log(f"[train] time limit reached after {n} scenes")
            break
        scene = sg.make_scene(s, cfg, device="cuda")
        ctx.set_scene(scene)
        srcs = list(range(1, len(scene.images)))
        d, nrm, c = ctx.patchmatch(0, srcs, sol["window"], sol["dilation"], sol["iters"], solver_params)
        X[n] = ctx.net_inputs(net, 0, srcs)
        tgt, mask = net.targets(d, nrm, c, args.max_cost)
        T[n] = tgt
        M[n] = mask
        D[n] = torch.tensor(scene.depth_range, dtype=torch.float32, device=dev)
        n += 1
        losses = train_steps(args.steps_per_scene, args.lr)
        history.append({"scene": s, "mask": float(mask.mean()), "loss": float(np.mean(losses))})
        if i % 10 == 0 or i == len(seeds) - 1:
            log(f"[train] scene {i + 1}/{len(seeds)} (seed {s}) mask {history[-1]['mask']:.3f} "
                f"loss {history[-1]['loss']:.4f} elapsed {time.time() - t0:.0f}s")
    final = []
    for k in range(0, args.final_steps, 100):
        final += train_steps(min(100, args.final_steps - k), args.lr_final)
        log(f"[train] final step {k + 100}: loss {np.mean(final[-100:]):.4f}")
    out = net.get_params()
    np.save(args.out, out)
    meta = {"scenes": n, "seeds": [seeds[0], seeds[n - 1]] if n else [], "config": cfg.__dict__, "solver": sol,
            "args": vars(args), "elapsed_s": time.time() - t0, "history": history,
            "final_loss": float(np.mean(final[-100:])) if final else None}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1, default=str)
    log(f"[train] wrote {args.out} after {n} scenes in {time.time() - t0:.0f}s")
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
