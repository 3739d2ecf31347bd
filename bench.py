"""Benchmark: pressure-Poisson solve to 1e-8 and matrix-free apply throughput
on one MI355X, for the 3D uniform level-7 workload (128^3 trilinear hexes,
2,146,689 nodes, phase field of 8 seeded tanh drops, Cn = 0.01, density ratio
1000, right-hand side b = M f with f a seeded sum of 8 cosine modes).

One step = set the phase field and solve the pressure system to a relative
residual of 1e-8 from x0 = 0 with multigrid-preconditioned CG in FP64
(set-up of the hierarchy for the new phase field included: exact fine
diagonal, fine stencil, Galerkin coarse operators, coarsest inverse; FP64
true-residual check), all inputs resident in HBM.  Jacobi-PCG, FP32-in-FP64
refinement and the learned preconditioner are reported as variants.

Prints one JSON line.  `python bench.py --profile-run` runs a short, fixed
sequence (a copy of known size, applies, one solve) meant to be wrapped by
rocprofv3.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import chns_inputs as ci  # noqa: E402

LEVEL = 7
CN = 0.01
RHO_P, RHO_M = 1.0, 1e-3
METRIC = "pressure-solve time to 1e-8 rel. residual & GDoF/s apply, plain vs learned+mixed"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (fma) x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6   # same lane count without packed FP32 (packed math is not used)
FP32_PACKED_PEAK_TFLOPS = 157.3  # the published FP32 vector peak (packed FP32)
# algorithmic work of one trilinear-hex pressure-Poisson leaf, sum-factorised:
# phase field to 8 Gauss points (72), 8 x (clamp 2 + fma 2 + reciprocal 9),
# 3 x (differences 4 + 2 transforms 24 + coefficient sums/products 8 + 2
# transforms 24 + scatter 8)
PP_FLOPS_PER_LEAF = 72 + 8 * 13 + 3 * (4 + 24 + 8 + 24 + 8)
PP_BYTES_PER_DOF = {8: 24, 4: 12}   # x and phi~ read once, y written once


def src_hash() -> str:
    h = hashlib.sha256()
    for f in ("apply.hip",):
        with open(os.path.join(ROOT, "paper_2107_05123_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def setup(torch):
    from paper_2107_05123_amd import Context, Mesh
    t0 = time.time()
    mesh = Mesh(dim=3, min_level=LEVEL, max_level=LEVEL, rule="uniform")
    t_mesh = time.time() - t0
    x_unit = ci.unit_coords(mesh.node_coords(), LEVEL)
    c, r = ci.drops(0)
    phi = ci.phi_drops(x_unit, c, r, CN)
    amps, waves = ci.rhs_modes(1)
    f = ci.rhs_field(x_unit, amps, waves)
    ctx = Context(mesh, Cn=CN, rho_plus=RHO_P, rho_minus=RHO_M)
    dev = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    phi_d = dev(phi)
    ctx.set_phase_field(phi_d)
    b = ctx.apply(ctx.MASS, dev(f))
    torch.cuda.synchronize()
    return mesh, ctx, phi_d, b, x_unit, phi, f, t_mesh


def time_applies(torch, ctx, x, n_warm=10, n_rep=100):
    """Median wall time of one apply from HIP events on the current stream."""
    for _ in range(n_warm):
        ctx.apply(ctx.PRESSURE, x)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_rep)]
    y = torch.empty_like(x)
    for a, b in ev:
        a.record()
        ctx.apply(ctx.PRESSURE, x, y)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def kernel_avg_ms(torch, ctx, x, tag, n_rep=50):
    """Average duration of one tagged launch group measured with HIP events
    that the library records on the stream it launches on."""
    y = torch.empty_like(x)
    ctx.apply(ctx.PRESSURE, x, y)
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    for _ in range(n_rep):
        ctx.apply(ctx.PRESSURE, x, y)
    torch.cuda.synchronize()
    ms, n = ctx.profile_read(tag)
    comb_ms, comb_n = ctx.profile_read("combine")
    ctx.profile(False)
    ctx.profile_reset()
    return ms / max(n, 1), comb_ms / max(comb_n, 1)


def solve_once(torch, ctx, phi_d, b, **kw):
    ctx.set_phase_field(phi_d)
    x = torch.zeros_like(b)
    x, st = ctx.solve_pressure(b, x, rtol=1e-8, **kw)
    return x, st


class RowSplit:
    """A CSR matrix whose products run as row blocks on a thread pool (scipy
    releases the GIL in its CSR kernels), so the oracle's own CG runs with a
    T-thread sparse product."""

    def __init__(self, A, threads):
        from concurrent.futures import ThreadPoolExecutor
        self.A, self.T = A, threads
        cuts = np.linspace(0, A.shape[0], threads + 1).astype(np.int64)
        self.blocks = [(int(cuts[i]), int(cuts[i + 1]), A[cuts[i]:cuts[i + 1]]) for i in range(threads)]
        self.pool = ThreadPoolExecutor(threads)
        self.shape = A.shape

    def __matmul__(self, v):
        out = np.empty(self.A.shape[0])

        def part(blk):
            lo, hi, Ab = blk
            out[lo:hi] = Ab @ v
        list(self.pool.map(part, self.blocks))
        return out

    def diagonal(self):
        return self.A.diagonal()


def host_threads():
    """Threads of this process's CPU share (at most 16, the share of one GPU on the pool's boxes)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(phi_nodes_lex, f_nodes_lex, pcg_iters):
    """Oracle timed on this host: mesh + CSR assembly + a bounded number of
    Jacobi-PCG iterations (the oracle's solver) on the same 128^3 problem,
    scaled to the iteration count that solver needs to reach 1e-8; once as it
    stands (one thread) and once with its CSR products split over the host's
    threads."""
    from oracle import fem, krylov, mesh as om
    t0 = time.time()
    m = om.uniform(3, LEVEL)
    side = 1 << LEVEL
    oc = m.indep_coords()
    # oracle node order -> lexicographic index (x fastest), the order of the inputs
    lex = oc[:, 0] + (side + 1) * (oc[:, 1] + (side + 1) * oc[:, 2])
    phi_o = phi_nodes_lex[lex]
    A = fem.pp_matrix(m, phi_o, RHO_P, RHO_M)
    M = fem.mass_matrix(m)
    b = M @ f_nodes_lex[lex]
    t_asm = time.time() - t0
    k_it = 20
    t1 = time.time()
    dinv = 1.0 / A.diagonal()
    x, it, hist = krylov.pcg(A, b, rtol=1e-30, max_it=k_it, M_inv_diag=dinv, singular=True)
    t_it = (time.time() - t1) / k_it
    t_spmv0 = time.time()
    for _ in range(5):
        A @ b
    t_spmv = (time.time() - t_spmv0) / 5
    est = t_asm + t_it * pcg_iters
    T = host_threads()
    At = RowSplit(A, T)
    At @ b
    t1 = time.time()
    krylov.pcg(At, b, rtol=1e-30, max_it=k_it, M_inv_diag=dinv, singular=True)
    t_it_T = (time.time() - t1) / k_it
    t_spmv0 = time.time()
    for _ in range(5):
        At @ b
    t_spmv_T = (time.time() - t_spmv0) / 5
    At.pool.shutdown()
    return {
        "value": est, "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle mesh + CSR assembly ({t_asm:.1f} s) and {k_it} Jacobi-PCG iterations "
                   f"({t_it * 1e3:.0f} ms each) on the full 128^3 problem, scaled to the {pcg_iters} Jacobi-PCG "
                   f"iterations that reach 1e-8; CSR SpMV {m.n_indep / t_spmv / 1e9:.4f} GDoF/s single-threaded scipy"),
        "spmv_gdof_s": m.n_indep / t_spmv / 1e9,
        "assembly_s": t_asm,
        "pcg_iter_s": t_it,
        "threads": {"value": t_asm + t_it_T * pcg_iters, "unit": "s", "cores": T,
                    "kind": "oracle, CSR products split over the host threads",
                    "sample": f"same assembly and {k_it} Jacobi-PCG iterations ({t_it_T * 1e3:.0f} ms each) with "
                              f"the CSR product in {T} row blocks on {T} threads, scaled to {pcg_iters} iterations",
                    "spmv_gdof_s": m.n_indep / t_spmv_T / 1e9, "pcg_iter_s": t_it_T},
    }


def load_traffic(tag):
    """HBM traffic per launch from a stored rocprofv3 PMC summary, only if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{tag}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("src_hash") != src_hash():
        return None
    return d.get("bytes_per_launch")


def apply_roofline(n_elems, n_dof, brick_ms, combine_ms, es=8):
    """Roofline entry of one whole pressure apply (brick kernel + combine,
    their average durations from the library's HIP events): algorithmic
    bytes (x, phi~ read, y written once: 24 B/DoF in FP64, 12 in FP32) and
    flops per launch over the apply's time, against HBM and the vector ALU.
    The brick kernel alone is kept as an extra entry."""
    flops = PP_FLOPS_PER_LEAF * n_elems
    nbytes = PP_BYTES_PER_DOF[es] * n_dof
    ms = brick_ms + combine_ms
    ach_flops = flops / (ms * 1e-3) / 1e12
    ach_gbs = nbytes / (ms * 1e-3) / 1e9
    peak_alu = FP64_PEAK_TFLOPS if es == 8 else FP32_PEAK_TFLOPS
    frac_alu = ach_flops / peak_alu
    frac_hbm = ach_gbs / HBM_PEAK_GBS
    traffic = load_traffic("pp_apply_fp64_l7" if es == 8 else "pp_apply_fp32_l7")
    # the bound is the resource whose roofline is lower at this intensity
    ridge = peak_alu * 1e12 / (HBM_PEAK_GBS * 1e9)
    if flops / nbytes >= ridge:
        roof = {"bound": "alu", "achieved": ach_flops, "peak": peak_alu, "unit": "TFLOP/s", "frac": frac_alu,
                "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": ach_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_hbm,
                "traffic": traffic}
    prec = "double" if es == 8 else "float"
    roof.update({"kernel": f"k_brick_o4<3,8,{prec},PP> + k_combine<{prec},1,0> (one apply)", "kernel_ms": ms,
                 "algorithmic_bytes_per_launch": nbytes, "algorithmic_flops_per_launch": flops,
                 "hbm_frac_algorithmic": frac_hbm, "alu_frac": frac_alu, "gdof_s": n_dof / (ms * 1e-3) / 1e9,
                 "brick_only": {"kernel_ms": brick_ms, "alu_frac": flops / (brick_ms * 1e-3) / 1e12 / peak_alu,
                                "hbm_frac_algorithmic": nbytes / (brick_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}})
    if es == 4:
        # the published FP32 vector peak counts packed FP32 (two per lane),
        # which this build does not use
        roof["alu_frac_vs_packed_peak"] = ach_flops / FP32_PACKED_PEAK_TFLOPS
    if traffic:
        roof["traffic_over_algorithmic"] = traffic / nbytes
    return roof


def summarize_stats(db, out_md, title, command, note, limit=30):
    """Markdown table of the top_kernels view of a rocprofv3 database."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                            f"limit {int(limit)}"))
    lines = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp, repository at $R):", "",
             f"    {command}", "", "The table is the `top_kernels` view of the rocpd database that command writes "
             "(durations in us).", note, "", "| calls | avg (us) | total (ms) | share | kernel |",
             "|---:|---:|---:|---:|---|"]
    for name, calls, tot, avg, pct in rows:
        lines.append(f"| {calls} | {avg:.2f} | {tot / 1e3:.3f} | {pct:.2f}% | `{name[:150]}` |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_pmc(fetch_csv, write_csv, out_prefix, commands):
    """HBM bytes per pressure apply (brick kernel + combine), FP64 and FP32,
    from FETCH_SIZE / WRITE_SIZE passes, calibrated on the 256 MiB device copy
    of the same run (the copy reads and writes 262144 KiB)."""
    import csv

    def per_kernel(path, key):
        with open(path) as fh:
            return [float(r["Counter_Value"]) for r in csv.DictReader(fh) if key in r["Kernel_Name"]]
    avg = lambda v: sum(v) / len(v) if v else 0.0
    ff = 262144.0 / max(per_kernel(fetch_csv, "copyBuffer"))
    fw = 262144.0 / max(per_kernel(write_csv, "copyBuffer"))
    out = {}
    for prec, es in (("double", 8), ("float", 4)):
        kb, kc = f"k_brick_o4<3, 8, {prec}, 0", f"k_combine<{prec}, 1, 0>"
        fb, wb = avg(per_kernel(fetch_csv, kb)) * ff * 1024, avg(per_kernel(write_csv, kb)) * fw * 1024
        fc, wc = avg(per_kernel(fetch_csv, kc)) * ff * 1024, avg(per_kernel(write_csv, kc)) * fw * 1024
        d = {"kernel": f"k_brick_o4<3,8,{prec},PP> + k_combine<{prec},1,0> (pressure-Poisson apply, 128^3)",
             "src_hash": src_hash(), "dispatches": len(per_kernel(fetch_csv, kb)),
             "fetch_factor": ff, "write_factor": fw,
             "calibration": "256 MiB device copy: FETCH_SIZE x fetch_factor and WRITE_SIZE x write_factor give "
                            "262144 KiB each",
             "bytes_per_launch": fb + wb + fc + wc,
             "brick_fetch_bytes": fb, "brick_write_bytes": wb, "combine_fetch_bytes": fc,
             "combine_write_bytes": wc, "commands": commands}
        name = f"{out_prefix}_fp{8 * es}_l7_pmc.json"
        with open(name, "w") as fh:
            json.dump(d, fh, indent=1)
        out[prec] = d
    return out


def profile_run(torch, with_solve=True, pc="jacobi"):
    """Fixed sequence for rocprofv3: copy of known size, FP64/FP32 applies, one solve."""
    mesh, ctx, phi_d, b, *_ = setup(torch)
    big = torch.empty(1 << 25, dtype=torch.float64, device="cuda")  # 256 MiB
    big2 = torch.empty_like(big)
    for _ in range(3):
        big2.copy_(big)
    x = torch.randn(mesh.n_nodes, dtype=torch.float64, device="cuda")
    for _ in range(20):
        ctx.apply(ctx.PRESSURE, x)
    x32 = x.float()
    for _ in range(20):
        ctx.apply(ctx.PRESSURE, x32)
    torch.cuda.synchronize()
    it = 0
    if with_solve:
        _, st = solve_once(torch, ctx, phi_d, b, pc=pc)
        it = st.iterations
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "done", "iterations": it, "copy_bytes": 2 * big.numel() * 8}))


def time_op(torch, ctx, op, x, n_warm=5, n_rep=30):
    """Median HIP-event time of one apply of `op`."""
    y = torch.empty_like(x)
    for _ in range(n_warm):
        ctx.apply(op, x, y)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_rep)]
    for a, b in ev:
        a.record()
        ctx.apply(op, x, y)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def chns_measure(torch, mesh, ctx, phi_d):
    """CHNS applies on the 128^3 mesh (VMS momentum, 3 DoF per node; CH Newton
    Jacobian, 2 DoF per node) and the per-step time of the 2D 64x64 drop
    (Re 100, We 1, Cn 0.02, density and viscosity ratios 10, dt 1e-3, two
    blocks per step)."""
    from paper_2107_05123_amd import Context, Mesh
    n = mesh.n_nodes
    g = torch.Generator(device="cuda").manual_seed(5)
    mu = 0.1 * torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    u = 0.3 * torch.randn(3 * n, dtype=torch.float64, device="cuda", generator=g)
    ctx.set_coefficients(ctx.MOMENTUM, [phi_d, mu, u])
    ctx.set_coefficients(ctx.CH_JACOBIAN, [phi_d, phi_d, u])
    ms_vp = time_op(torch, ctx, ctx.MOMENTUM, torch.randn(3 * n, dtype=torch.float64, device="cuda", generator=g))
    ms_ch = time_op(torch, ctx, ctx.CH_JACOBIAN, torch.randn(2 * n, dtype=torch.float64, device="cuda",
                                                             generator=g))
    out = {"momentum_apply": {"ms": ms_vp, "gdof_s": 3 * n / (ms_vp * 1e-3) / 1e9},
           "ch_jacobian_apply": {"ms": ms_ch, "gdof_s": 2 * n / (ms_ch * 1e-3) / 1e9}}
    # 2D drop, 64 x 64
    m2 = Mesh(dim=2, min_level=6, max_level=6, rule="uniform")
    x2 = ci.unit_coords(m2.node_coords(), 6)
    c2 = Context(m2, Re=100.0, We=1.0, Cn=0.02, Fr=1.0, rho_plus=1.0, rho_minus=0.1, eta_plus=1.0,
                 eta_minus=0.1, dt=1e-3)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    phi2 = dev(ci.phi_drop2d(x2, cn=0.02))
    n2 = m2.n_nodes
    st = {"u": dev(np.zeros(2 * n2)), "u_prev": dev(np.zeros(2 * n2)), "p": dev(np.zeros(n2)), "phi": phi2,
          "mu": c2.initial_mu(phi2)}
    c2.advance_step(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [c2.advance_step(st) for _ in range(10)]
    torch.cuda.synchronize()
    out["step_2d_64"] = {"ms_per_step": 1e3 * (time.perf_counter() - t0) / 10,
                         "newton": stats[-1]["newton"], "ch_gmres_it": stats[-1]["ch_iterations"],
                         "vp_gmres_it": stats[-1]["vp_iterations"], "pp_cg_it": stats[-1]["pp_iterations"],
                         "vu_cg_it": stats[-1]["vu_iterations"], "mass": stats[-1]["mass"],
                         "energy": stats[-1]["energy"]}
    return out


def profile_unet(torch):
    """Fixed sequence for rocprofv3: 20 forward passes of the shipped network
    on the 128^3 node grid (after one warm-up)."""
    mesh, ctx, phi_d, b, *_ = setup(torch)
    with open(os.path.join(ROOT, "paper_2107_05123_amd", "weights", "unet_uniform_l7_rho1000.bin"), "rb") as fh:
        ctx.pc_load(fh.read())
    r = b - b.mean()
    out = ctx.pc_forward(phi_d, r, crop=128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        ctx.pc_forward(phi_d, r, crop=128, out=out)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "unet done", "forward_ms": (time.perf_counter() - t0) / 20 * 1e3}))


def profile_chns(torch):
    """Fixed sequence for rocprofv3: CHNS applies on 128^3, three steps of the
    2D 64x64 drop, three U-Net forward passes on a 128^3 crop."""
    mesh, ctx, phi_d, b, *_ = setup(torch)
    n = mesh.n_nodes
    g = torch.Generator(device="cuda").manual_seed(5)
    mu = 0.1 * torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    u = 0.3 * torch.randn(3 * n, dtype=torch.float64, device="cuda", generator=g)
    ctx.set_coefficients(ctx.MOMENTUM, [phi_d, mu, u])
    ctx.set_coefficients(ctx.CH_JACOBIAN, [phi_d, phi_d, u])
    for _ in range(5):
        ctx.apply(ctx.MOMENTUM, u)
        ctx.apply(ctx.CH_JACOBIAN, u[:2 * n])
    wpath = os.path.join(ROOT, "paper_2107_05123_amd", "weights", "unet_uniform_l7_rho1000.bin")
    with open(wpath, "rb") as fh:
        ctx.pc_load(fh.read())
    r = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    for _ in range(3):
        ctx.pc_forward(phi_d, r, crop=128)
    torch.cuda.synchronize()
    from paper_2107_05123_amd import Context, Mesh
    m2 = Mesh(dim=2, min_level=6, max_level=6, rule="uniform")
    x2 = ci.unit_coords(m2.node_coords(), 6)
    c2 = Context(m2, Re=100.0, We=1.0, Cn=0.02, Fr=1.0, rho_plus=1.0, rho_minus=0.1, eta_plus=1.0,
                 eta_minus=0.1, dt=1e-3)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    phi2 = dev(ci.phi_drop2d(x2, cn=0.02))
    n2 = m2.n_nodes
    st = {"u": dev(np.zeros(2 * n2)), "u_prev": dev(np.zeros(2 * n2)), "p": dev(np.zeros(n2)), "phi": phi2,
          "mu": c2.initial_mu(phi2)}
    for _ in range(3):
        c2.advance_step(st)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "chns done"}))


def uniform_apply(torch, level):
    """Pressure apply on a finer uniform octree (level 8: 256^3 leaves, eight
    waves per SIMD slot in turn): FP64 and FP32 throughput and the brick /
    combine split by the library's HIP events."""
    from paper_2107_05123_amd import Context, Mesh
    mesh = Mesh(dim=3, min_level=level, max_level=level, rule="uniform")
    x = ci.unit_coords(mesh.node_coords(), level)
    ctx = Context(mesh, Cn=CN, rho_plus=RHO_P, rho_minus=RHO_M)
    c, r = ci.drops(0)
    ctx.set_phase_field(torch.tensor(ci.phi_drops(x, c, r, CN), dtype=torch.float64, device="cuda"))
    n = mesh.n_nodes
    xr = torch.tensor(ci.normal_vector(0, n), dtype=torch.float64, device="cuda")
    out = {"workload": f"3D uniform octree level {level} ({1 << level}^3 Q1 hex, {n:,} nodes), 8 seeded drops, "
                       "density ratio 1000", "n_elems": mesh.n_elems, "n_dof": n}
    for prec, v in (("fp64", xr), ("fp32", xr.float())):
        ms = time_applies(torch, ctx, v)
        k, comb = kernel_avg_ms(torch, ctx, v, "pp_brick_" + prec)
        out[prec] = {"gdof_s": n / (ms * 1e-3) / 1e9, "ms": ms, "brick_ms": k, "combine_ms": comb}
    return out


def adaptive_workload(torch, lmax):
    """Adaptive octree, levels 5..lmax refined within 3 Cn of the rising-bubble
    interface (R 0.15, centre (0.5, 0.3, 0.5), Cn 0.01), density ratio 1000:
    apply throughput and pressure solves to 1e-8, FP64 plain vs FP32 applies
    inside FP64 iterative refinement."""
    from paper_2107_05123_amd import Context, Mesh
    t0 = time.time()
    mesh = Mesh(dim=3, min_level=5, max_level=lmax, rule="sphere_band", centres=[(0.5, 0.3, 0.5)], radii=[0.15],
                band=3 * CN)
    t_mesh = time.time() - t0
    print(f"# mesh built in {t_mesh:.1f} s: {mesh.summary()['n_elems']} leaves", file=sys.stderr, flush=True)
    x_unit = ci.unit_coords(mesh.node_coords(), lmax)
    ctx = Context(mesh, Cn=CN, rho_plus=RHO_P, rho_minus=RHO_M)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    phi_d = dev(ci.phi_bubble(x_unit, cn=CN))
    ctx.set_phase_field(phi_d)
    amps, waves = ci.rhs_modes(1)
    b = ctx.apply(ctx.MASS, dev(ci.rhs_field(x_unit, amps, waves)))
    n = mesh.n_nodes
    xr = torch.tensor(ci.normal_vector(0, n), dtype=torch.float64, device="cuda")
    ms64 = time_applies(torch, ctx, xr)
    ms32 = time_applies(torch, ctx, xr.float())
    out = {"workload": f"3D adaptive octree levels 5-{lmax}, band 3 Cn around the rising bubble (Cn 0.01), "
                       "density ratio 1000, pressure Poisson",
           "n_elems": mesh.n_elems, "n_dof": n, "n_hanging": mesh.summary()["n_hanging"],
           "host_mesh_build_s": t_mesh,
           "apply_gdof_s": {"fp64": n / (ms64 * 1e-3) / 1e9, "fp32": n / (ms32 * 1e-3) / 1e9,
                            "fp64_ms": ms64, "fp32_ms": ms32},
           "hbm_frac_algorithmic_fp64": PP_BYTES_PER_DOF[8] * n / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "solves": {}}
    for name, kw in (("gmg_pcg_fp64", dict(pc="gmg")), ("gmg_pcg_mixed_ir", dict(pc="gmg", mode="mixed")),
                     ("jacobi_pcg_fp64", dict(pc="jacobi", max_it=40000)),
                     ("jacobi_pcg_mixed_ir", dict(pc="jacobi", mode="mixed", max_it=40000)),
                     ("jacobi_pcg_mixed_ru", dict(pc="jacobi", mode="mixed_ru", inner_rtol=1e-2, max_it=40000))):
        solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sv = solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        out["solves"][name] = {"s": time.perf_counter() - t1, "iterations": sv.iterations,
                               "outer": sv.outer_iterations, "rel_residual": sv.rel_residual,
                               "setup_ms": sv.ms_setup}
        print(f"# {name}: {out['solves'][name]}", file=sys.stderr, flush=True)
    # learned preconditioner through the uniform level-7 grid (the shipped
    # weights; the grid transfers are built on the host at the first solve)
    wpath = os.path.join(ROOT, "paper_2107_05123_amd", "weights", "unet_uniform_l7_rho1000.bin")
    with open(wpath, "rb") as fh:
        ctx.pc_load(fh.read())
    t1 = time.perf_counter()
    solve_once(torch, ctx, phi_d, b, pc="learned", learned_every=8)
    torch.cuda.synchronize()
    out["learned_grid_setup_s"] = time.perf_counter() - t1
    for name, kw in (("learned_fcg_every8_fp64", dict(pc="learned", learned_every=8, max_it=40000)),
                     ("learned_fcg_every8_mixed_ir", dict(pc="learned", learned_every=8, mode="mixed",
                                                          max_it=40000))):
        solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sv = solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        out["solves"][name] = {"s": time.perf_counter() - t1, "iterations": sv.iterations,
                               "outer": sv.outer_iterations, "rel_residual": sv.rel_residual,
                               "setup_ms": sv.ms_setup, "fallback_to_jacobi": sv.fallback}
        print(f"# {name}: {out['solves'][name]}", file=sys.stderr, flush=True)
    return out


# held-out instance seeds timed in the benchmark line (the full 0-99
# evaluation is train_pc.py --eval-only ... --eval-seeds 0-99)
LEARNED_SEEDS = 10


def learned_distribution(torch, ctx, x_unit, seeds):
    """Jacobi-PCG against flexible CG with the network every 8th iteration on
    held-out instances of the 128^3 drop family (phase field and right-hand
    side of each seed evaluated on the GPU), each solve timed after a warm-up
    of the same instance."""
    from paper_2107_05123_amd.train_pc import GpuInputs, instance_gpu
    gin = GpuInputs(torch, x_unit)
    rows = []
    for seed in seeds:
        _, b_s = instance_gpu(gin, ctx, seed)
        row = {"seed": seed}
        for name, kw in (("jacobi_pcg_fp64", dict(pc="jacobi")),
                         ("learned_fcg_every8_fp64", dict(pc="learned", learned_every=8))):
            ctx.solve_pressure(b_s, **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, st = ctx.solve_pressure(b_s, **kw)
            torch.cuda.synchronize()
            row[name] = (time.perf_counter() - t1, st.iterations)
        rows.append(row)
    out = {"seeds": f"{seeds[0]}-{seeds[-1]}", "note": "seeds 0-99: profiles/learned_pc_uniform_l7_seeds0-99.md"}
    for name in ("jacobi_pcg_fp64", "learned_fcg_every8_fp64"):
        ms = np.array([r[name][0] for r in rows]) * 1e3
        it = np.array([r[name][1] for r in rows])
        out[name] = {"ms_median": float(np.median(ms)), "ms_min": float(ms.min()), "ms_max": float(ms.max()),
                     "iterations_median": float(np.median(it)), "iterations_min": int(it.min()),
                     "iterations_max": int(it.max())}
    out["learned_faster_on"] = int(sum(r["learned_fcg_every8_fp64"][0] < r["jacobi_pcg_fp64"][0] for r in rows))
    return out


def bubble_steps(torch, lmax, nsteps, ch_pc="block", restart=16, vp_pc="jacobi", modes=("fp64", "mixed"),
                 remesh_every=0, max_seconds=0.0):
    """Projection time steps of the 3D rising bubble (density ratio 1000,
    viscosity ratio 100, Re 35, We 10, Cn 0.005, dt 5e-4) on the adaptive
    octree of levels 5..lmax refined within 3 Cn of the interface; with
    remesh_every = K > 0 the mesh is rebuilt around |phi| <= 0.95 after every
    K steps and the state carried over by the intergrid transfer.  With
    max_seconds > 0 no new step starts after that much wall time since the
    start (the steps taken are reported)."""
    from paper_2107_05123_amd import Context, Mesh, Transfer
    cn = 0.005
    t0 = time.time()
    mesh = Mesh(dim=3, min_level=5, max_level=lmax, rule="sphere_band", centres=[(0.5, 0.3, 0.5)], radii=[0.15],
                band=3 * cn)
    t_mesh = time.time() - t0
    print(f"# mesh built in {t_mesh:.1f} s: {mesh.n_elems} leaves, {mesh.n_nodes} nodes", file=sys.stderr, flush=True)
    x_unit = ci.unit_coords(mesh.node_coords(), lmax)
    prm = dict(Re=35.0, We=10.0, Cn=cn, Fr=1.0, rho_plus=1.0, rho_minus=1e-3, eta_plus=1.0, eta_minus=1e-2, dt=5e-4)
    ctx = Context(mesh, **prm)
    print(f"# context ready ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    n = mesh.n_nodes
    phi = dev(ci.phi_bubble(x_unit, cn=cn))
    st = {"u": dev(np.zeros(3 * n)), "u_prev": dev(np.zeros(3 * n)), "p": dev(np.zeros(n)), "phi": phi,
          "mu": ctx.initial_mu(phi)}
    torch.cuda.synchronize()
    print(f"# initial state ready ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    out = {"workload": f"3D rising bubble, adaptive levels 5-{lmax} (band 3 Cn, Cn 0.005), density ratio 1000, "
                       "viscosity ratio 100, Re 35, We 10, dt 5e-4",
           "ch_preconditioner": ch_pc, "vp_preconditioner": vp_pc, "gmres_restart": restart,
           "n_elems": mesh.n_elems, "n_nodes": n, "host_mesh_build_s": t_mesh, "steps": [], "remesh": []}
    for mode in modes:
        for k in range(nsteps):
            if max_seconds > 0 and time.time() - t0 > max_seconds:
                out["stopped_at_time_limit"] = {"mode": mode, "steps_done": k}
                break
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s = ctx.advance_step(st, pp_pc="gmg", pp_mode=mode, ch_pc=ch_pc, restart=restart, vp_pc=vp_pc)
            torch.cuda.synchronize()
            s["wall_s"] = time.perf_counter() - t1
            s["pressure_mode"] = mode
            s["n_elems"] = mesh.n_elems
            out["steps"].append(s)
            print(f"# step {k} ({mode}): {s}", file=sys.stderr, flush=True)
            if remesh_every > 0 and (k + 1) % remesh_every == 0:
                # remesh around |phi| <= 0.95 and carry the state over
                r = {"after_step": k, "old_elems": mesh.n_elems}
                t2 = time.perf_counter()
                phi_h = st["phi"].cpu().numpy()
                new = mesh.remesh(phi_h, 5, 0.95)
                r["host_remesh_s"] = time.perf_counter() - t2
                t2 = time.perf_counter()
                tr = Transfer(mesh, new)
                r["host_transfer_build_s"] = time.perf_counter() - t2
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                st = {"u": tr.apply(st["u"], n_fields=3), "u_prev": tr.apply(st["u_prev"], n_fields=3),
                      "p": tr.apply(st["p"]), "phi": tr.apply(st["phi"]), "mu": tr.apply(st["mu"])}
                torch.cuda.synchronize()
                r["device_transfer_ms"] = (time.perf_counter() - t2) * 1e3
                del ctx
                t2 = time.perf_counter()
                ctx = Context(new, **prm)
                torch.cuda.synchronize()
                r["context_s"] = time.perf_counter() - t2
                mesh = new
                r["new_elems"] = mesh.n_elems
                r["new_nodes"] = mesh.n_nodes
                out["remesh"].append(r)
                print(f"# remesh: {r}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true", help="leave out the adaptive (levels 5-10) key")
    ap.add_argument("--adaptive-level", type=int, default=10, help="finest level of the adaptive key")
    ap.add_argument("--profile-run", nargs="?", const="full", default=None,
                    help="fixed sequence for rocprofv3; 'applies' skips the solve (for counter passes), "
                         "'gmg' solves with multigrid CG, 'chns' runs the CHNS applies, steps and network passes, "
                         "'unet' 20 network forward passes")
    ap.add_argument("--workload", default="uniform_l7", choices=("uniform_l7", "adaptive", "bubble_steps"),
                    help="uniform_l7: the benchmark line; adaptive: levels 5..--max-level band mesh solves; "
                         "bubble_steps: projection steps of the 3D rising bubble")
    ap.add_argument("--max-level", type=int, default=10)
    ap.add_argument("--max-seconds", type=float, default=0.0,
                    help="bubble_steps: start no step after this much wall time (0: no limit)")
    ap.add_argument("--restart", type=int, default=20,
                    help="bubble_steps: GMRES restart length (short cycles keep the Gram-Schmidt cost of the "
                         "large CH and momentum bases down)")
    ap.add_argument("--ch-pc", default="schur", choices=("block", "schur"),
                    help="bubble_steps: preconditioner of the Cahn-Hilliard GMRES (2x2 node-block Jacobi, or the "
                         "block-triangular multigrid Schur-complement preconditioner)")
    ap.add_argument("--vp-pc", default="gmg", choices=("jacobi", "gmg"),
                    help="bubble_steps: preconditioner of the velocity-prediction GMRES (Jacobi, or multigrid "
                         "V-cycles of the scalar mass + viscous operator per component)")
    ap.add_argument("--remesh-every", type=int, default=0,
                    help="bubble_steps: rebuild the mesh around |phi| <= 0.95 after every K steps (0: never)")
    ap.add_argument("--pp-modes", default="fp64,mixed",
                    help="bubble_steps: pressure solve modes to step with, in order (comma-separated)")
    ap.add_argument("--summarize-stats", nargs=5, metavar=("DB", "OUT_MD", "TITLE", "COMMAND", "NOTE"),
                    help="write the kernel-statistics table of a rocprofv3 database (no GPU needed)")
    ap.add_argument("--summarize-pmc", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_PREFIX", "CMD1", "CMD2"),
                    help="write the HBM-traffic summaries of the FP64 and FP32 pressure applies (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_stats:
        db, out, title, cmd, note = args.summarize_stats
        summarize_stats(db, out, title, cmd, note)
        return
    if args.summarize_pmc:
        fc, wc, out, c1, c2 = args.summarize_pmc
        print(json.dumps(summarize_pmc(fc, wc, out, [c1, c2]), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (it would shard by "
              "contiguous Morton ranges of bricks, with halo exchange of shared nodes)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "adaptive":
        print(json.dumps(adaptive_workload(torch, args.max_level)))
        return
    if args.workload == "bubble_steps":
        print(json.dumps(bubble_steps(torch, args.max_level, args.steps, args.ch_pc, args.restart, args.vp_pc,
                                      tuple(args.pp_modes.split(",")), args.remesh_every, args.max_seconds)))
        return
    if args.profile_run == "chns":
        profile_chns(torch)
        return
    if args.profile_run == "unet":
        profile_unet(torch)
        return
    if args.profile_run:
        profile_run(torch, with_solve=args.profile_run != "applies",
                    pc="gmg" if args.profile_run == "gmg" else "jacobi")
        return
    mesh, ctx, phi_d, b, x_unit, phi, f, t_mesh = setup(torch)
    n = mesh.n_nodes

    # ---- warm-up and timed steps (plain FP64 GMG-PCG)
    for _ in range(args.warmup):
        solve_once(torch, ctx, phi_d, b, pc="gmg")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        _, st = solve_once(torch, ctx, phi_d, b, pc="gmg")
        stats.append(st)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = 1e3 * t_steps / args.steps
    st = stats[-1]

    # ---- variants (each timed once after one warm-up)
    variants = {"gmg_pcg_fp64": {"s": ms_per_step / 1e3, "iterations": st.iterations,
                                 "rel_residual": st.rel_residual, "setup_ms": st.ms_setup}}
    for name, kw in (("gmg_pcg_mixed_ir", dict(pc="gmg", mode="mixed", inner_rtol=1e-4)),
                     ("jacobi_pcg_fp64", dict(pc="jacobi")),
                     ("jacobi_pcg_mixed_ir", dict(pc="jacobi", mode="mixed", inner_rtol=1e-4)),
                     ("jacobi_pcg_mixed_ru", dict(pc="jacobi", mode="mixed_ru", inner_rtol=1e-2))):
        solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sv = solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        variants[name] = {"s": time.perf_counter() - t1, "iterations": sv.iterations,
                          "outer": sv.outer_iterations, "rel_residual": sv.rel_residual,
                          "setup_ms": sv.ms_setup}

    # ---- learned preconditioner (trained weights shipped with the package)
    wpath = os.path.join(ROOT, "paper_2107_05123_amd", "weights", "unet_uniform_l7_rho1000.bin")
    with open(wpath, "rb") as fh:
        ctx.pc_load(fh.read())
    for name, kw in (("learned_fcg_every8_fp64", dict(pc="learned", learned_every=8)),
                     ("learned_fcg_every8_mixed_ir", dict(pc="learned", learned_every=8, mode="mixed",
                                                          inner_rtol=1e-4)),
                     ("learned_fcg_every8_mixed_ru", dict(pc="learned", learned_every=8, mode="mixed_ru",
                                                          inner_rtol=1e-2)),
                     ("learned_fcg_every_iteration_fp64", dict(pc="learned"))):
        solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sv = solve_once(torch, ctx, phi_d, b, **kw)
        torch.cuda.synchronize()
        variants[name] = {"s": time.perf_counter() - t1, "iterations": sv.iterations,
                          "outer": sv.outer_iterations, "rel_residual": sv.rel_residual,
                          "setup_ms": sv.ms_setup, "fallback_to_jacobi": sv.fallback}
    learned_seeds = learned_distribution(torch, ctx, x_unit, range(LEARNED_SEEDS))
    ctx.set_phase_field(phi_d)

    # ---- apply throughput and the dominant kernel's roofline
    xr = torch.tensor(ci.normal_vector(0, n), dtype=torch.float64, device="cuda")
    ms64 = time_applies(torch, ctx, xr)
    ms32 = time_applies(torch, ctx, xr.float())
    k64, comb64 = kernel_avg_ms(torch, ctx, xr, "pp_brick_fp64")
    k32, comb32 = kernel_avg_ms(torch, ctx, xr.float(), "pp_brick_fp32")
    roof = apply_roofline(mesh.n_elems, n, k64, comb64)
    roof32 = apply_roofline(mesh.n_elems, n, k32, comb32, es=4)
    E = mesh.n_elems

    out = {
        "metric": METRIC,
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D uniform octree level 7 (128^3 Q1 hex, 2,146,689 nodes), pressure Poisson "
                               "-div((1/rho(phi)) grad p), 8 seeded tanh drops (Cn 0.01), density ratio 1000, "
                               "multigrid-preconditioned CG (FP64) to 1e-8 from x0 = 0, set-up included",
                   "n_dof": n, "n_elems": E},
        "apply_gdof_s": {"fp64": n / (ms64 * 1e-3) / 1e9, "fp32": n / (ms32 * 1e-3) / 1e9,
                         "fp64_ms": ms64, "fp32_ms": ms32,
                         "brick_fp64_ms": k64, "combine_fp64_ms": comb64,
                         "brick_fp32_ms": k32, "combine_fp32_ms": comb32},
        "roofline": roof,
        "roofline_fp32": roof32,
        "variants": variants, "learned_seeds": learned_seeds,
        "iterations": st.iterations,
        "rel_residual": st.rel_residual,
        "host_mesh_build_s": t_mesh,
        "chns": chns_measure(torch, mesh, ctx, phi_d),
    }
    out["apply_uniform_l8"] = uniform_apply(torch, 8)
    if not args.no_adaptive:
        out["adaptive"] = adaptive_workload(torch, args.adaptive_level)
    if not args.no_cpu_baseline:
        lex = np.arange(n)  # uniform meshes are numbered lexicographically, x fastest
        out["cpu_baseline"] = cpu_baseline(phi[lex], f[lex], variants["jacobi_pcg_fp64"]["iterations"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
