"""Training and evaluation of the learned preconditioner on the GPU.

Every arithmetic step runs in libapcloud.so: the training data (apc_learn_data),
the forward/backward pass (apc_mlp_loss_grad), the optimiser (apc_mlp_adam) and
the BF16 inference that installs M (apc_set_learned_precond).  This module only
draws the seeded clouds and probe vectors and sequences the calls.

The network maps 48 features of a row of the assembled Poisson operator to the
41 weights of row i of M (the pattern of row i of the operator: the diagonal and
up to 40 stencil nodes, the nearest 40 of a fourth-order row) as
m_i = (e_0 + o_i) / d_i, so an all-zero output layer is Jacobi.  The loss is the
left approximate-inverse residual ||m_i^T A - e_i^T||^2 estimated with Gaussian
probe vectors.  Second- and fourth-order operators get a network each, trained
on clouds of their own order.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import apcloud as apc

TRAIN_SEEDS = tuple(range(4000, 4200))
HELD_OUT_SEEDS = tuple(range(5000, 5020))
_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "learned_params.npy")

# per GFD order: the cloud recipe, training and held-out seeds, parameter file
RECIPES = {
    2: dict(workload="beam_halo_1e5", train=TRAIN_SEEDS, held_out=HELD_OUT_SEEDS,
            params=PARAMS_PATH),
    4: dict(workload="beam_halo_k4_3e4", train=tuple(range(6000, 6200)),
            held_out=tuple(range(7000, 7020)),
            params=os.path.join(_HERE, "learned_params_k4.npy")),
}


def params_path(order: int) -> str:
    return RECIPES[order]["params"]


def _workload(name):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from workloads import CONFIGS, beam_halo
    return CONFIGS[name], beam_halo


def make_cloud(seed, workload="beam_halo_1e5", precision=apc.APC_MIXED):
    """A cloud of the named workload recipe drawn with another seed, assembled."""
    import torch
    cfg, beam_halo = _workload(workload)
    xyz = beam_halo(cfg["N"], seed=seed, sigma=cfg["sigma"], halo_frac=cfg["halo_frac"])
    cloud = apc.Cloud(torch.from_numpy(xyz).cuda(), order=cfg["order"], c=cfg["c"],
                      max_depth=cfg["max_depth"], precision=precision)
    cloud.assemble_gfd()
    return cloud


def training_data(seeds=TRAIN_SEEDS, K=32, workload="beam_halo_1e5", probe_seed=7,
                  precision=apc.APC_MIXED, log=None):
    """Features and quadratic loss data of every interior row of the clouds."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(probe_seed)
    feats, quads = [], []
    for k, sd in enumerate(seeds):
        if log and k % 50 == 0:
            log(f"training data: cloud {k} of {len(seeds)}")
        cloud = make_cloud(sd, workload, precision)
        Z = torch.randn((K, cloud.n + cloud.nb), dtype=torch.float64, device="cuda",
                        generator=gen)
        f, q = cloud.learn_data(Z)
        feats.append(f)
        quads.append(q)
        torch.cuda.synchronize()
        cloud.close()
    return torch.cat(feats), torch.cat(quads)


SAFEGUARD_PROBES = 16


def probes(cloud, K=SAFEGUARD_PROBES, seed=0):
    """K Gaussian probe vectors for the install's safeguard (device, float64)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    return torch.randn((K, cloud.n + cloud.nb), dtype=torch.float64, device="cuda",
                       generator=gen)


def init_params(seed=0):
    """He-initialised hidden layers, zero output layer (starts at Jacobi)."""
    import torch
    rng = np.random.default_rng(seed)
    IN, H, O = apc.MLP_IN, apc.MLP_HID, apc.MLP_OUT
    parts = [rng.standard_normal(IN * H) * np.sqrt(2.0 / IN), np.zeros(H),
             rng.standard_normal(H * H) * np.sqrt(2.0 / H), np.zeros(H),
             np.zeros(H * O), np.zeros(O)]
    P = np.concatenate(parts).astype(np.float32)
    assert P.size == apc.MLP_NPARAM
    return torch.from_numpy(P).cuda()


def train(feat, quad, steps=3000, batch=4096, lr=1e-3, seed=0, params=None, log_every=250,
          log=None):
    """Adam on minibatches of rows; returns the parameters and the loss history."""
    import torch
    P = init_params(seed) if params is None else params.clone()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 1)
    nrow = feat.shape[0]
    grad = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(1, steps + 1):
        rows = torch.randint(0, nrow, (batch,), device="cuda", generator=gen, dtype=torch.int32)
        apc.mlp_loss_grad(P, feat, quad, rows, grad=grad, loss=loss)
        apc.mlp_adam(P, m, v, grad, step, lr)
        if step == 1 or step % log_every == 0 or step == steps:
            hist.append((step, float(loss.item())))
            if log:
                log(f"step {step} loss {hist[-1][1]:.6f}")
    return P, hist


def full_loss(P, feat, quad, chunk=1 << 18):
    """Mean loss over all rows (forward of apc_mlp_loss_grad in chunks)."""
    import torch
    tot = 0.0
    n = feat.shape[0]
    for a in range(0, n, chunk):
        rows = torch.arange(a, min(n, a + chunk), dtype=torch.int32, device="cuda")
        L, _ = apc.mlp_loss_grad(P, feat, quad, rows)
        tot += float(L.item()) * rows.numel()
    return tot / n


def evaluate(P, seeds=HELD_OUT_SEEDS, workload="beam_halo_1e5", tol=1e-8,
             precision=apc.APC_MIXED, maxit=20000):
    """Poisson solve of every held-out cloud with Jacobi and with the learned M
    (same right-hand side from the deposit); iterations and solve times."""
    import torch
    out = []
    for sd in seeds:
        cloud = make_cloud(sd, workload, precision)
        _, rho_t, _ = cloud.deposit(tol=1e-10, maxit=4000)
        b = rho_t[:cloud.n].contiguous()
        res = {"seed": sd, "n": cloud.n}
        for name, pc in (("jacobi", apc.APC_PRECOND_JACOBI), ("learned", apc.APC_PRECOND_LEARNED)):
            if pc == apc.APC_PRECOND_LEARNED:
                t0 = time.perf_counter()
                cloud.set_learned_precond(P, probes(cloud, seed=sd))
                res["install_ms"] = (time.perf_counter() - t0) * 1e3
            # one untimed solve, then the timed one
            cloud.solve(b, tol=tol, maxit=maxit, precond=pc)
            phi, st = cloud.solve(b, tol=tol, maxit=maxit, precond=pc)
            res[name] = dict(iters=st["iters"], ms=st["ms"], status=st["status"],
                             precond_used=st["precond_used"],
                             rel_resid_true=st["rel_resid_true"])
            res[name + "_phi"] = phi[:cloud.n].clone()
        torch.cuda.synchronize()
        cloud.close()
        out.append(res)
    return out


def summarize(results):
    it_j = np.array([r["jacobi"]["iters"] for r in results], dtype=float)
    it_l = np.array([r["learned"]["iters"] for r in results], dtype=float)
    ms_j = np.array([r["jacobi"]["ms"] for r in results])
    ms_l = np.array([r["learned"]["ms"] for r in results])
    return dict(clouds=len(results), iters_jacobi=float(it_j.mean()), iters_learned=float(it_l.mean()),
                iter_ratio=float(it_j.sum() / it_l.sum()), ms_jacobi=float(ms_j.mean()),
                ms_learned=float(ms_l.mean()), time_ratio=float(ms_j.sum() / ms_l.sum()),
                fallbacks=int(sum(r["learned"]["precond_used"] != apc.APC_PRECOND_LEARNED
                                  for r in results)))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--order", type=int, default=2, choices=sorted(RECIPES))
    ap.add_argument("--train-clouds", type=int, default=200)
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-clouds", type=int, default=20)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    rec = RECIPES[args.order]
    out_path = args.out or rec["params"]
    import torch

    def log(msg):
        print(f"[learned] {msg}", file=sys.stderr, flush=True)

    apc.load_library()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    feat, quad = training_data(rec["train"][:args.train_clouds], K=args.probes,
                               workload=rec["workload"], log=log)
    log(f"training data: {feat.shape[0]} rows from {args.train_clouds} clouds "
        f"({time.perf_counter() - t0:.1f} s)")
    P0 = init_params(0)
    l0 = full_loss(P0, feat, quad)
    t0 = time.perf_counter()
    P, hist = train(feat, quad, steps=args.steps, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    l1 = full_loss(P, feat, quad)
    log(f"loss {l0:.5f} (Jacobi) -> {l1:.5f} in {t_train:.1f} s")
    np.save(out_path, P.cpu().numpy())
    res = evaluate(P, rec["held_out"][:args.eval_clouds], workload=rec["workload"])
    s = summarize(res)
    s.update(order=args.order, loss_jacobi=l0, loss_trained=l1, train_s=t_train,
             train_rows=int(feat.shape[0]))
    print(json.dumps(s), flush=True)


if __name__ == "__main__":
    main()
