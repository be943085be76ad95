#!/usr/bin/env python3
"""Benchmark of the EBE hot path on one MI355X.

Workload (the EBE-matvec configuration): unit cube, 64^3 hexes x 6 = 1,572,864
straight 10-node tetrahedra, 2,146,689 nodes (6.44M DOF), interior corners
jittered by U(-0.2, 0.2) h, three horizontal layers (E = 1, 3, 8; nu = 0.25,
0.27, 0.30), seeded N(0, 1) input vectors.

A step is one y = K [x_1 .. x_16] product in FP32 (ebe_matvec: the element
patch kernel plus the shared-node pass), the form the mixed-precision solver
spends its time in.  `value` is DOF x RHS processed per second (GDOF.RHS/s)
with inputs resident in HBM.  The other (dtype, n) combinations, the
roofline of the product, the CPU oracle on a bounded sample, and (unless
--no-solver) whole solves per second of the multi-case crust workload are
reported on the same JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published MI355X vector ALU peaks: FP32 157.3 TFLOP/s (256 CU x 4 SIMD x 16
# lanes x 2 flop x 2.4 GHz x 2, the last factor being packed two-wide FP32
# FMA), FP64 78.6 TFLOP/s.  The library is compiled with packed FP32 instructions off, so
# plain FP32 FMA peaks at 78.6 as well; both fractions are reported.
ALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
ALU_PEAK_UNPACKED_TFLOPS = 78.6
# Floating-point operations (FMA = 2) of the matrix-free element product per
# (element, case), as written in p2_element.h: corner outer products 48, their
# sum 18, per-corner strain and stress coefficients 330, corner forces 108,
# edge forces 252 (scaled stress sums 54, two tensor-vector products per edge
# 198): 756.  Element geometry (once per element) is not counted.
FLOPS_PER_ELEM_RHS = 756


def product_bytes(N, Nv, E, n, p):
    """Compulsory bytes of one EBE product: read x and write y once, the
    connectivity (10 int32), corner coordinates (3 doubles) and one material
    pair per element."""
    return 2 * 3 * N * n * p + 40 * E + 24 * Nv + 2 * E * p


def source_hash():
    h = hashlib.sha256()
    for f in ("ebe_kernels.hip", "p2_element.h", "patches.cpp", "ebe_internal.h"):
        with open(os.path.join(ROOT, "paper_1710_08679_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(tag):
    """HBM bytes per product from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "ebe_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("products", {}).get(tag)
    return None if k is None else float(k["fetch_bytes"] + k["write_bytes"])


def time_launches(fn, steps, warmup, torch):
    """Average milliseconds of fn over `steps` calls, timed with HIP events on
    torch's current stream (the stream the library launches on)."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        fn(i)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def cpu_baseline(mesh, n, n_elem_sample):
    """The oracle's EBE product (Eq. (3) by definition) on the first
    n_elem_sample elements, scaled to the whole mesh."""
    from oracle import fem
    from paper_1710_08679_amd import meshgen
    x = meshgen.random_vectors(meshgen.rng_for(2, 99), mesh.n_nodes, n)
    sl = slice(0, n_elem_sample)
    t0, c0 = time.perf_counter(), time.process_time()
    fem.ebe_apply(mesh.xyz, mesh.conn[sl], mesh.young[sl], mesh.poisson[sl], x)
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    rate = (n_elem_sample / mesh.n_elem) * mesh.n_dof * n / wall / 1e9
    return {"value": rate, "unit": "GDOF*RHS/s", "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
            "sample": f"oracle EBE product (dense K_e by 4-point quadrature, scatter by bincount) over the first "
                      f"{n_elem_sample} of {mesh.n_elem} elements of the same mesh, FP64, n={n}; {wall:.1f} s "
                      f"wall; rate scaled by the element fraction",
            "host_cpus": os.cpu_count()}


def solver_block(torch, ebe, meshgen, modes=("mixed_mg3", "mixed_mg2", "fp64_mg2", "fp64_pcge")):
    """Solves per second of the multi-case crust workload: 96x96x48 hexes x 6
    = 2,654,208 tetrahedra, 16 dislocation-pair cases, to 1e-8."""
    m = meshgen.crust_mesh(96, 96, 48)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    gm = ebe.Mesh.from_generated(m)
    fd = torch.from_numpy(f).cuda()
    fixed = torch.from_numpy(m.fixed.astype(bool)).cuda()
    out = {"workload": "crust 96x96x48 hexes x 6 tets, 3 layers, 16 cases, tol 1e-8 (unsquared, max over cases)",
           "elements": m.n_elem, "dof": m.n_dof, "runs": []}
    ref = None
    table = {"mixed_mg3": (ebe.PREC_MG3, ebe.MODE_MIXED), "fp64_mg3": (ebe.PREC_MG3, ebe.MODE_FP64),
             "mixed_mg2": (ebe.PREC_MG2, ebe.MODE_MIXED), "fp64_mg2": (ebe.PREC_MG2, ebe.MODE_FP64),
             "fp64_pcge": (ebe.PREC_PCGE, ebe.MODE_FP64)}
    for name in modes:
        precond, mode = table[name]
        torch.cuda.synchronize()
        tw = time.perf_counter()
        gm.solve(fd, precond=precond, mode=mode, tol=1e-8)  # warm-up: block Jacobi, level-2 set-up, workspace
        torch.cuda.synchronize()
        t_first = time.perf_counter() - tw
        t0 = time.perf_counter()
        u, st = gm.solve(fd, precond=precond, mode=mode, tol=1e-8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = fd.clone()
        r[fixed] = 0
        Ku = gm.matvec(u, apply_bc=True)
        res = float((torch.linalg.vector_norm((r - Ku).reshape(-1, 16), dim=0)
                     / torch.linalg.vector_norm(r.reshape(-1, 16), dim=0)).max())
        entry = {"mode": name, "seconds": dt, "first_solve_seconds": t_first, "solves_per_s": 16.0 / dt,
                 "outer_iters": st["outer_iters"],
                 "inner_iters": st["inner_iters"], "max_rel_res": st["max_rel_res"], "fp64_rel_res": res}
        if ref is None:
            ref = u.clone()
        else:
            entry["rel_diff_vs_first"] = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(u))
        out["runs"].append(entry)
        print(f"# solver {name}: {dt:.3f} s, {st}", file=sys.stderr, flush=True)
    return out


FORM_NAMES = {0: "gather", 1: "staged", 2: "pipelined", 3: "assembled"}


def adjoint_block(torch, ebe, meshgen, steps, warmup):
    """The adjoint workload: 64x64x32 hexes x 6 = 786,432 tets, lognormal moduli,
    4 cases: the element-gradient kernel g_e = -sum_c lam_c,e^T (K_e/E_e) u_c,e
    in FP64 and FP32, and one full dMisfit/dE (forward solve, adjoint solve,
    kernel) through torch.autograd with default solver options (FP64 outer)."""
    from paper_1710_08679_amd.autograd import surface_misfit
    m = meshgen.adjoint_mesh(64, 64, 32)
    gm = ebe.Mesh.from_generated(m)
    n = 4
    out = {"workload": "adjoint 64x64x32 hexes x 6 tets, lognormal E, 4 cases", "elements": m.n_elem, "runs": []}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        u = torch.randn((m.n_nodes, 3, n), dtype=torch.float64, device="cuda").to(dt)
        lam = torch.randn((m.n_nodes, 3, n), dtype=torch.float64, device="cuda").to(dt)
        g = torch.empty((m.n_elem,), dtype=dt, device="cuda")
        t = time_launches(lambda i: gm.adjoint_grad(u, lam, out=g), steps, warmup, torch)
        out["runs"].append({"kernel": "adjoint_grad", "dtype": name, "ms": t,
                            "gelem_case_per_s": m.n_elem * n / (t * 1e-3) / 1e9,
                            "input_gb_per_s": 2 * 3 * m.n_nodes * n * (8 if name == "f64" else 4) / (t * 1e-3) / 1e9})
        print(f"# adjoint kernel {name} n={n}: {t:.3f} ms, {out['runs'][-1]['gelem_case_per_s']:.1f} Gelem*case/s",
              file=sys.stderr, flush=True)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(4, 3), nrhs=n)
    S = torch.from_numpy(meshgen.top_surface_dofs(m)).cuda()
    d = 1e-3 * torch.randn((S.shape[0], n), dtype=torch.float64, device="cuda")
    fd = torch.from_numpy(f).cuda()
    pd = torch.from_numpy(m.poisson).cuda()
    for rep_i in range(2):  # the first one sets up the level-2 operator and workspace
        E = torch.from_numpy(m.young).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = surface_misfit(E, gm, pd, fd, S, d)
        loss.backward()
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
    out["runs"].append({"kernel": "misfit + gradient (two solves + kernel)", "dtype": "mixed solves, f64 kernel",
                        "seconds": dt_s})
    print(f"# adjoint misfit + gradient: {dt_s:.3f} s", file=sys.stderr, flush=True)
    return out


def batch_block(torch, ebe, meshgen, n_mesh, with_big):
    """Batched uneven serving-size set: n_mesh crust meshes with log-uniform
    element counts in [5e4, 2e6] and 1..16 cases each (optionally plus the
    128x128x64 mesh with 16 cases), mixed MG2 to 1e-8, solved as one batch
    and then one after another."""
    grids, nrhs = meshgen.batch_sizes(meshgen.rng_for(5, 0), n_mesh=n_mesh)
    if with_big:
        grids.append((128, 128, 64))
        nrhs.append(16)
    gms, fs = [], []
    for k, (gr, n) in enumerate(zip(grids, nrhs)):
        m = meshgen.crust_mesh(*gr)
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(5, 100 + k), nrhs=n)
        gms.append(ebe.Mesh.from_generated(m))
        fs.append(torch.from_numpy(f).cuda())
        print(f"# batch mesh {k}: grid {gr}, {m.n_elem} tets, {n} cases", file=sys.stderr, flush=True)
    opts = ebe.default_opts(tol=1e-8)
    ebe.batch_solve(gms, fs, opts=opts)  # warm-up: block Jacobi set-up, workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st_b = ebe.batch_solve(gms, fs, opts=opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    st_s = [gm.solve(f, opts=opts)[1] for gm, f in zip(gms, fs)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    cases = int(sum(nrhs))
    out = {"workload": f"{n_mesh} crust meshes, log-uniform 5e4..2e6 tets, 1..16 cases each"
                       + (" + 128x128x64 (16 cases)" if with_big else "") + ", mixed MG2 to 1e-8",
           "n_mesh": len(grids), "elements_total": int(sum(g.n_elem for g in gms)), "cases_total": cases,
           "batch_seconds": tb, "sequential_seconds": ts, "speedup": ts / tb,
           "solves_per_s_batch": cases / tb, "solves_per_s_sequential": cases / ts,
           "max_rel_res": max(s["max_rel_res"] for s in st_b),
           "all_converged": all(s["status"] == ebe.OK for s in st_b + st_s)}
    print(f"# batch: {tb:.3f} s batched vs {ts:.3f} s one by one, {cases} cases", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--variants", default="f64:1,f64:4,f64:16,f32:1,f32:4,f32:16",
                    help="comma list of dtype:n products to time")
    ap.add_argument("--no-solver", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--solver-modes", default="mixed_mg3,mixed_mg2,fp64_mg2,fp64_pcge")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-elems", type=int, default=100000)
    ap.add_argument("--batch", type=int, default=0, metavar="N_MESH",
                    help="also time a batch of N_MESH uneven crust meshes against one-by-one solves")
    ap.add_argument("--batch-big", action="store_true", help="add the 128x128x64 mesh to the batch")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1710_08679_amd import ebe, meshgen

    ebe.load()
    torch.cuda.set_device(0)
    g = args.grid
    mesh = meshgen.matvec_mesh(g)
    gm = ebe.Mesh.from_generated(mesh)
    N, Nv, E = mesh.n_nodes, mesh.n_vertices, mesh.n_elem
    print(f"# workload {g}^3 x 6: E={E} N={N} DOF={3 * N}", file=sys.stderr, flush=True)

    tdt = {"f64": (torch.float64, 8), "f32": (torch.float32, 4)}
    variants = []
    for spec in args.variants.split(","):
        name, n = spec.split(":")
        n = int(n)
        dt, p = tdt[name]
        vec_bytes = 3 * N * n * p
        sets = max(3, int(np.ceil(1.1e9 / (2 * vec_bytes))))  # > 1 GB of x/y: no reuse through the 256 MB MALL
        tms = gm.autotune(0, dt, n)  # keeps the fastest product form for (dtype, n) on this mesh
        xs = [torch.randn((N, 3, n), dtype=torch.float64, device="cuda").to(dt) for _ in range(sets)]
        ys = [torch.empty((N, 3, n), dtype=dt, device="cuda") for _ in range(sets)]
        t_op = time_launches(lambda i: gm.matvec(xs[i % sets], out=ys[i % sets]), args.steps, args.warmup, torch)
        B = product_bytes(N, Nv, E, n, p)
        rec = {"dtype": name, "nrhs": n, "ms": t_op, "form": FORM_NAMES[gm.form(0, dt, n)],
               "autotune_ms": {FORM_NAMES[f]: t for f, t in enumerate(tms) if t >= 0},
               "gdof_rhs_per_s": 3 * N * n / (t_op * 1e-3) / 1e9,
               "hbm_frac": B / (t_op * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "alu_frac": E * n * FLOPS_PER_ELEM_RHS / (t_op * 1e-3) / 1e12 / ALU_PEAK_TFLOPS[name]}
        variants.append(rec)
        print(f"# {name} n={n} ({rec['form']}; tuning ms: " + " / ".join(f"{FORM_NAMES[f]} {t:.3f}" for f, t in enumerate(tms) if t >= 0) + "): "
              f"{t_op:.3f} ms, {rec['gdof_rhs_per_s']:.1f} GDOF*RHS/s, "
              f"HBM {rec['hbm_frac']:.2%}, ALU {rec['alu_frac']:.2%}", file=sys.stderr, flush=True)
        del xs, ys
        torch.cuda.empty_cache()

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    # timed region of the headline step: FP32, 16 cases, y = K x, in the form
    # the autotuner picked on this mesh
    n, dt, p = 16, torch.float32, 4
    if gm.form(0, dt, n) == -1 or "f32:16" not in args.variants.split(","):
        gm.autotune(0, dt, n)
    form = FORM_NAMES[gm.form(0, dt, n)]
    sets = 3
    xs = [torch.randn((N, 3, n), dtype=torch.float64, device="cuda").to(dt) for _ in range(sets)]
    ys = [torch.empty((N, 3, n), dtype=dt, device="cuda") for _ in range(sets)]
    for i in range(args.warmup):
        gm.matvec(xs[i % sets], out=ys[i % sets])
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for i in range(args.steps):
        gm.matvec(xs[i % sets], out=ys[i % sets])
    b.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ms_events = a.elapsed_time(b) / args.steps
    value = 3 * N * n / (ms * 1e-3) / 1e9
    del xs, ys
    torch.cuda.empty_cache()

    t = ms_events * 1e-3
    B = product_bytes(N, Nv, E, n, p)
    F = E * n * FLOPS_PER_ELEM_RHS
    hbm = {"bound": "hbm", "achieved": B / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": B / t / 1e9 / HBM_PEAK_GBS}
    alu = {"bound": "alu", "achieved": F / t / 1e12, "peak": ALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
           "frac": F / t / 1e12 / ALU_PEAK_TFLOPS["f32"],
           "frac_of_unpacked_fp32_peak": F / t / 1e12 / ALU_PEAK_UNPACKED_TFLOPS}
    roof, alt = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    traffic = load_traffic(f"f32:16:{form}")
    roof["traffic"] = traffic
    roof["kernel"] = (f"EBE product FP32 n=16, {form} form: "
                      + {"gather": "k_ebe_patch<float,16,2,false,false>", "staged": "k_ebe_patch<float,16,2,true,false>",
                         "pipelined": "k_ebe_patch_pipe<float,16,2,false>"}[form] + " + k_reduce_shared<float,16>")
    roof["ms_per_launch"] = ms_events
    roof["algorithmic_bytes"] = B
    roof["algorithmic_flops"] = F
    if traffic is not None:
        roof["traffic_over_algorithmic"] = traffic / B

    line = {"metric": "EBE matvec GDOF*RHS/s (FP32, 16 cases) and % HBM peak; PCG solves/s mixed vs FP64",
            "value": value, "unit": "GDOF*RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"EBE matvec, unit cube {g}^3 hexes x 6 tets, jitter 0.2h, 3 layers, 16 cases",
                       "elements": E, "nodes": N, "dof": 3 * N, "nrhs": 16},
            "roofline": roof, "roofline_alt": alt, "variants": variants}
    if not args.no_solver:
        line["solver"] = solver_block(torch, ebe, meshgen, args.solver_modes.split(","))
    if not args.no_adjoint:
        line["adjoint"] = adjoint_block(torch, ebe, meshgen, args.steps, args.warmup)
    if args.batch > 0:
        line["batch"] = batch_block(torch, ebe, meshgen, args.batch, args.batch_big)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(mesh, 16, args.cpu_elems)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
