"""Train the learned pressure preconditioner on the GPU.

Samples come from the 3D uniform level-7 family (128^3 hexes, eight seeded
tanh drops with Cn = 0.01, density ratio 1000): for every instance seed the
right-hand side b = M f (f a seeded sum of cosine modes) is solved to 1e-11
with multigrid-preconditioned CG, and the triples (phase field, r_k, e_k) are
taken along the Jacobi-PCG trajectory from x0 = 0 after k iterations
(r_k = b - A x_k, e_k = x* - x_k).  Default objective: on the full node grid
the preconditioner output z = rms(r) K Net(coef, r / rms(r)) is scored by its
A-norm error (e - z)^T A (e - z) / e^T r, which is what conjugate gradients
needs of a preconditioner (alternative: mean squared error against
e / (rms(r) K) on random 64^3 crops with mirror augmentation).  K is the
mean of rms(e) / rms(r) over the samples.  Every kernel (solves, applies,
network, backpropagation, Adam) runs in libchns.

    python -m paper_2107_05123_amd.train_pc --out weights.bin [--instances N]
        [--steps S] [--eval-seeds 0,1,2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import chns_inputs as ci  # noqa: E402

LEVEL = 7
CN = 0.01
RHO_P, RHO_M = 1.0, 1e-3


def log(msg):
    print(msg, flush=True)


def make_context(torch):
    from paper_2107_05123_amd import Context, Mesh
    mesh = Mesh(dim=3, min_level=LEVEL, max_level=LEVEL, rule="uniform")
    ctx = Context(mesh, Cn=CN, rho_plus=RHO_P, rho_minus=RHO_M)
    x_unit = ci.unit_coords(mesh.node_coords(), LEVEL)
    return mesh, ctx, x_unit


def instance(torch, ctx, x_unit, seed):
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    c, r = ci.drops(seed)
    phi = dev(ci.phi_drops(x_unit, c, r, CN))
    amps, waves = ci.rhs_modes(seed)
    ctx.set_phase_field(phi)
    b = ctx.apply(ctx.MASS, dev(ci.rhs_field(x_unit, amps, waves)))
    b = b - b.mean()
    return phi, b


def samples(torch, ctx, x_unit, seeds, ks):
    out = []
    for s in seeds:
        phi, b = instance(torch, ctx, x_unit, s)
        xs, st = ctx.solve_pressure(b, rtol=1e-11, pc="gmg")
        for k in ks:
            if k == 0:
                xk = torch.zeros_like(b)
            else:
                xk, _ = ctx.solve_pressure(b, rtol=1e-30, max_it=k, pc="jacobi", raise_on_noconv=False)
            rk = b - ctx.apply(ctx.PRESSURE, xk)
            ek = xs - xk
            out.append((phi, rk, ek))
        log(f"instance {s}: gmg iterations {st.iterations}, {len(ks)} samples")
    return out


def evaluate(torch, ctx, x_unit, seeds):
    rows = []
    for s in seeds:
        phi, b = instance(torch, ctx, x_unit, s)
        row = {"seed": s}
        for name, kw in (("jacobi", dict(pc="jacobi")), ("gmg", dict(pc="gmg")),
                         ("learned_every8", dict(pc="learned", learned_every=8)),
                         ("learned_every8_mixed", dict(pc="learned", learned_every=8, mode="mixed"))):
            ctx.solve_pressure(b, **kw)  # warm-up (graphs, buffers)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = ctx.solve_pressure(b, **kw)
            torch.cuda.synchronize()
            row[name] = {"s": time.perf_counter() - t0, "iterations": st.iterations, "fallback": st.fallback,
                         "rel_residual": st.rel_residual}
        log(json.dumps(row))
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--instances", type=int, default=24)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--ks", default="0,8,32,128")
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--objective", default="anorm", choices=("anorm", "crop_mse"))
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--crop", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--omega", type=float, default=0.6, help="Jacobi damping around the network (0: network alone)")
    ap.add_argument("--eval-seeds", default="0,1")
    ap.add_argument("--max-seconds", type=float, default=600.0)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t_start = time.time()
    mesh, ctx, x_unit = make_context(torch)
    ks = [int(k) for k in args.ks.split(",")]
    data = samples(torch, ctx, x_unit, range(args.first_seed, args.first_seed + args.instances), ks)
    ratios = [float(torch.sqrt((e * e).mean()) / torch.sqrt((r * r).mean())) for _, r, e in data]
    K = float(np.mean(ratios))
    log(f"{len(data)} samples in {time.time() - t_start:.1f} s, K = {K:.4g}")
    ctx.pc_init(seed=args.init_seed, out_scale=K, omega=args.omega)
    rng = np.random.default_rng(args.init_seed)
    side = 1 << LEVEL
    hi = side + 1 - args.crop
    t_train = time.time()
    ema = None
    for step in range(args.steps):
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps)) + 1e-5
        idx = rng.integers(0, len(data), args.batch)
        origins = [tuple(int(v) for v in rng.integers(0, hi + 1, 3)) for _ in idx]
        flips = [int(f) for f in rng.integers(0, 8, args.batch)]
        loss = ctx.pc_train_step([data[i][0] for i in idx], [data[i][1] for i in idx], [data[i][2] for i in idx],
                                 origins, args.crop, flips=flips, lr=lr, objective=args.objective)
        ema = loss if ema is None else 0.95 * ema + 0.05 * loss
        if step % 25 == 0 or step == args.steps - 1:
            log(f"step {step} loss {loss:.4g} ema {ema:.4g} lr {lr:.2e} "
                f"({(time.time() - t_train) / (step + 1) * 1e3:.1f} ms/step)")
        if time.time() - t_start > args.max_seconds:
            log(f"time limit reached after {step + 1} steps")
            break
    blob = ctx.pc_save()
    with open(args.out, "wb") as fh:
        fh.write(blob)
    log(f"wrote {args.out} ({len(blob)} bytes)")
    if args.eval_seeds:
        evaluate(torch, ctx, x_unit, [int(s) for s in args.eval_seeds.split(",")])


if __name__ == "__main__":
    main()
