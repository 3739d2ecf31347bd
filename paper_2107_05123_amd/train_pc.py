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

With --stream every training step draws fresh instances (seeds first-seed,
first-seed + 1, ...; one trajectory sample each, k drawn from --ks), so the
network sees instances * 1 samples without storing them; the phase field and
right-hand side of an instance are evaluated on the GPU from its seeded
drop and mode parameters.  --eval-seeds a-b evaluates every seed in the
range against Jacobi- and multigrid-PCG and writes per-seed rows and a
summary with --eval-out.
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


class GpuInputs:
    """Seeded instances evaluated on the GPU (the same recipe as chns_inputs:
    phi = -1 + sum_d [1 + tanh((R_d - |x - c_d|)/(sqrt2 Cn))], f = sum_k a_k
    prod_d cos(w_kd pi x_d)), to keep host time out of streamed training."""

    def __init__(self, torch, x_unit):
        self.torch = torch
        self.x = torch.tensor(x_unit, dtype=torch.float64, device="cuda")

    def phi(self, seed):
        t = self.torch
        c, r = ci.drops(seed)
        out = t.full((self.x.shape[0],), -1.0, dtype=t.float64, device="cuda")
        for cc, rr in zip(c, r):
            dist = t.sqrt(((self.x - t.tensor(cc, dtype=t.float64, device="cuda")) ** 2).sum(1))
            out += 1.0 + t.tanh((float(rr) - dist) / (ci.SQRT2 * CN))
        return out

    def rhs_field(self, seed):
        t = self.torch
        amps, waves = ci.rhs_modes(seed)
        out = t.zeros(self.x.shape[0], dtype=t.float64, device="cuda")
        for a, w in zip(amps, waves):
            term = t.full_like(out, float(a))
            for d in range(3):
                term = term * t.cos(float(w[d]) * math.pi * self.x[:, d])
            out += term
        return out


def instance_gpu(gin, ctx, seed):
    phi = gin.phi(seed)
    ctx.set_phase_field(phi)
    b = ctx.apply(ctx.MASS, gin.rhs_field(seed))
    return phi, b - b.mean()


def exact_solution(ctx, b):
    """x* = A^-1 b by multigrid CG to 1e-11, or None when the solve stops
    above 1e-9 (at density ratio 1000 a few instances reach the FP64 floor of
    the pressure system before 1e-11)."""
    xs, st = ctx.solve_pressure(b, rtol=1e-11, pc="gmg", raise_on_noconv=False)
    return xs if st.rel_residual <= 1e-9 else None


def sample_at(torch, ctx, b, xs, k):
    if k == 0:
        xk = torch.zeros_like(b)
    else:
        xk, _ = ctx.solve_pressure(b, rtol=1e-30, max_it=k, pc="jacobi", raise_on_noconv=False)
    return b - ctx.apply(ctx.PRESSURE, xk), xs - xk


def samples(torch, ctx, x_unit, seeds, ks):
    out = []
    for s in seeds:
        phi, b = instance(torch, ctx, x_unit, s)
        xs, st = ctx.solve_pressure(b, rtol=1e-11, pc="gmg", raise_on_noconv=False)
        if st.rel_residual > 1e-9:
            log(f"instance {s}: multigrid stopped at {st.rel_residual:.2e}; skipped")
            continue
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


def evaluate(torch, ctx, x_unit, seeds, gin=None):
    rows = []
    for s in seeds:
        phi, b = instance_gpu(gin, ctx, s) if gin is not None else instance(torch, ctx, x_unit, s)
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
    ap.add_argument("--eval-seeds", default="0,1", help="comma list or a range a-b (inclusive)")
    ap.add_argument("--eval-out", default=None, help="JSON file for the evaluation rows and summary")
    ap.add_argument("--eval-only", default=None, help="evaluate this weight blob instead of training")
    ap.add_argument("--stream", action="store_true", help="fresh instances every step (see the module text)")
    ap.add_argument("--max-seconds", type=float, default=600.0)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t_start = time.time()
    mesh, ctx, x_unit = make_context(torch)
    gin = GpuInputs(torch, x_unit)
    if args.eval_only:
        with open(args.eval_only, "rb") as fh:
            ctx.pc_load(fh.read())
        run_eval(torch, ctx, x_unit, gin, args)
        return
    ks = [int(k) for k in args.ks.split(",")]
    if args.stream:
        train_stream(torch, ctx, gin, ks, args, t_start)
        run_eval(torch, ctx, x_unit, gin, args)
        return
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
    run_eval(torch, ctx, x_unit, gin, args)


def parse_seeds(text):
    if not text:
        return []
    if "-" in text:
        a, b = (int(v) for v in text.split("-"))
        return list(range(a, b + 1))
    return [int(v) for v in text.split(",")]


def run_eval(torch, ctx, x_unit, gin, args):
    seeds = parse_seeds(args.eval_seeds)
    if not seeds:
        return
    rows = evaluate(torch, ctx, x_unit, seeds, gin)
    names = [k for k in rows[0] if k != "seed"]
    summ = {}
    for k in names:
        it = np.array([r[k]["iterations"] for r in rows], dtype=float)
        tm = np.array([r[k]["s"] for r in rows]) * 1e3
        summ[k] = {"iterations_median": float(np.median(it)), "iterations_min": float(it.min()),
                   "iterations_max": float(it.max()), "ms_median": float(np.median(tm)), "ms_min": float(tm.min()),
                   "ms_max": float(tm.max()), "fallbacks": int(sum(r[k]["fallback"] for r in rows)),
                   "max_rel_residual": float(max(r[k]["rel_residual"] for r in rows))}
    log(json.dumps({"summary": summ, "seeds": [seeds[0], seeds[-1]], "n": len(seeds)}))
    if args.eval_out:
        with open(args.eval_out, "w") as fh:
            json.dump({"summary": summ, "rows": rows}, fh, indent=1)


def train_stream(torch, ctx, gin, ks, args, t_start):
    """Online training: every step takes args.batch fresh instances (next
    seeds), solves each to 1e-11 with multigrid CG, and draws one Jacobi-PCG
    trajectory sample (k from ks) per instance."""
    rng = np.random.default_rng(args.init_seed)
    # output scale K from a few instances
    ratios = []
    for s in range(args.first_seed, args.first_seed + 4):
        phi, b = instance_gpu(gin, ctx, s)
        xs = exact_solution(ctx, b)
        if xs is None:
            continue
        for k in ks:
            r, e = sample_at(torch, ctx, b, xs, k)
            ratios.append(float(torch.sqrt((e * e).mean()) / torch.sqrt((r * r).mean())))
    K = float(np.mean(ratios))
    ctx.pc_init(seed=args.init_seed, out_scale=K, omega=args.omega)
    log(f"K = {K:.4g}; streaming {args.instances} instances in batches of {args.batch}")
    steps = max(1, args.instances // args.batch)
    seed = args.first_seed
    t_train = time.time()
    ema = None
    skipped = 0
    for step in range(steps):
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / steps)) + 1e-5
        batch = []
        while len(batch) < args.batch:
            phi, b = instance_gpu(gin, ctx, seed)
            seed += 1
            xs = exact_solution(ctx, b)
            if xs is None:
                skipped += 1
                continue
            r, e = sample_at(torch, ctx, b, xs, int(ks[rng.integers(0, len(ks))]))
            batch.append((phi, r, e))
        loss = ctx.pc_train_step([t[0] for t in batch], [t[1] for t in batch], [t[2] for t in batch], None,
                                 args.crop, flips=None, lr=lr, objective=args.objective)
        ema = loss if ema is None else 0.97 * ema + 0.03 * loss
        if step % 50 == 0 or step == steps - 1:
            log(f"step {step} (seed {seed}) loss {loss:.4g} ema {ema:.4g} lr {lr:.2e} "
                f"({(time.time() - t_train) / (step + 1) * 1e3:.1f} ms/step)")
        if time.time() - t_start > args.max_seconds:
            log(f"time limit reached after {step + 1} steps ({seed - args.first_seed} instances)")
            break
    blob = ctx.pc_save()
    with open(args.out, "wb") as fh:
        fh.write(blob)
    log(f"wrote {args.out} ({len(blob)} bytes); {seed - args.first_seed} instances "
        f"({skipped} skipped: multigrid stopped above 1e-9)")


if __name__ == "__main__":
    main()
