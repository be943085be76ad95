#!/usr/bin/env python3
"""Benchmark of the EBE hot path on one MI355X.

Workload (the EBE-matvec configuration): unit cube, 64^3 hexes x 6 = 1,572,864
straight 10-node tetrahedra, 2,146,689 nodes (6.44M DOF), interior corners
jittered by U(-0.2, 0.2) h, three horizontal layers (E = 1, 3, 8; nu = 0.25,
0.27, 0.30), seeded N(0, 1) input vectors.

A step is one y = K [x_1 .. x_16] product in FP32 (ebe_matvec, clearing pass
included), the form the mixed-precision solver spends its time in.  `value`
is DOF x RHS processed per second (GDOF.RHS/s) with inputs resident in HBM.
The other (dtype, n) combinations, the kernel roofline, the CPU oracle on a
bounded sample, and (unless --no-solver) whole solves per second of the
multi-case crust workload are reported on the same JSON line.
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
# Vector ALU peak with plain (non-packed) FP32 / FP64 FMA:
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s for both.
ALU_PEAK_TFLOPS = 78.6
# Floating-point operations of the matrix-free element product per (element,
# case), counting an FMA as 2 (see p2_element.h): strain coefficients 447,
# forces 354.
FLOPS_PER_ELEM_RHS = 801


def kernel_bytes(N, Nv, E, n, p):
    """Compulsory bytes of one EBE product: read x and write y once, the
    connectivity (10 int32), corner coordinates (3 doubles) and one material
    pair per element."""
    return 2 * 3 * N * n * p + 40 * E + 24 * Nv + 2 * E * p


def source_hash():
    h = hashlib.sha256()
    for f in ("ebe_kernels.hip", "p2_element.h"):
        with open(os.path.join(ROOT, "paper_1710_08679_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_tag):
    """HBM traffic per dispatch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "ebe_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_tag)
    return None if k is None else float(k["fetch_bytes"] + k["write_bytes"])


def time_launches(fn, steps, warmup, torch):
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
    return a.elapsed_time(b) / steps  # ms


def cpu_baseline(mesh, n, n_elem_sample):
    """The oracle's EBE product (Eq. (3) by definition) on the first
    n_elem_sample elements, scaled to the whole mesh."""
    import numpy as np
    from oracle import fem
    from paper_1710_08679_amd import meshgen
    x = meshgen.random_vectors(meshgen.rng_for(2, 99), mesh.n_nodes, n)
    sl = slice(0, n_elem_sample)
    t0, c0 = time.perf_counter(), time.process_time()
    fem.ebe_apply(mesh.xyz, mesh.conn[sl], mesh.young[sl], mesh.poisson[sl], x)
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    frac = n_elem_sample / mesh.n_elem
    rate = frac * mesh.n_dof * n / wall / 1e9
    return {"value": rate, "unit": "GDOF*RHS/s", "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
            "sample": f"oracle EBE product (dense K_e by quadrature, scatter by bincount) over the first "
                      f"{n_elem_sample} of {mesh.n_elem} elements, FP64, n={n}; {wall:.1f} s wall, "
                      f"rate scaled by the element fraction",
            "host_cpus": os.cpu_count()}


def solver_block(torch, ebe, meshgen, steps_solver=1):
    """Solves per second of the multi-case crust workload: 96x96x48 hexes x 6
    = 2,654,208 tetrahedra, 16 dislocation-pair cases, to 1e-8."""
    import numpy as np
    m = meshgen.crust_mesh(96, 96, 48)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    gm = ebe.Mesh.from_generated(m)
    fd = torch.from_numpy(f).cuda()
    out = {"workload": "crust 96x96x48 hexes x 6 tets, 3 layers, 16 cases, tol 1e-8 (unsquared)",
           "elements": m.n_elem, "dof": m.n_dof, "runs": []}
    ref = None
    for name, precond, mode in (("mixed_mg2", ebe.PREC_MG2, ebe.MODE_MIXED),
                                ("fp64_mg2", ebe.PREC_MG2, ebe.MODE_FP64),
                                ("fp64_pcge", ebe.PREC_PCGE, ebe.MODE_FP64)):
        u, st = gm.solve(fd, precond=precond, mode=mode, tol=1e-8)  # warm-up (sets up blocks/workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps_solver):
            u, st = gm.solve(fd, precond=precond, mode=mode, tol=1e-8)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps_solver
        # independent FP64 residual with the FP64 EBE product
        r = fd.clone()
        r[torch.from_numpy(m.fixed.astype(bool)).cuda()] = 0
        Ku = gm.matvec(u, apply_bc=True)
        res = float(torch.linalg.vector_norm((r - Ku).reshape(-1, 16), dim=0).max()
                    / torch.linalg.vector_norm(r.reshape(-1, 16), dim=0).max())
        entry = {"mode": name, "seconds": dt, "solves_per_s": 16.0 / dt, "outer_iters": st["outer_iters"],
                 "inner_iters": st["inner_iters"], "max_rel_res": st["max_rel_res"], "fp64_rel_res": res}
        if ref is None:
            ref = u.clone()
        else:
            entry["rel_diff_vs_mixed"] = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(u))
        out["runs"].append(entry)
        print(f"# solver {name}: {dt:.3f} s, {st}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--no-solver", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-elems", type=int, default=40000)
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

    variants = []
    head = None
    for dt, p, name in ((torch.float64, 8, "f64"), (torch.float32, 4, "f32")):
        for n in (1, 4, 16):
            vec_bytes = 3 * N * n * p
            sets = max(3, int(np.ceil(1.1e9 / (2 * vec_bytes))))  # > 1 GB of x/y: no reuse from the 256 MB MALL
            xs = [torch.randn((N, 3, n), dtype=torch.float64, device="cuda").to(dt) for _ in range(sets)]
            ys = [torch.zeros((N, 3, n), dtype=dt, device="cuda") for _ in range(sets)]
            # kernel only: y += K x (no clearing pass), rotating buffer sets
            t_k = time_launches(lambda i: gm.matvec_add(xs[i % sets], ys[i % sets]), args.steps, args.warmup, torch)
            # the user-visible operation: y = K x (clearing pass + kernel)
            t_op = time_launches(lambda i: gm.matvec(xs[i % sets], out=ys[i % sets]), args.steps, args.warmup,
                                 torch)
            B = kernel_bytes(N, Nv, E, n, p)
            rec = {"dtype": name, "nrhs": n, "ms_matvec": t_op, "ms_kernel": t_k,
                   "gdof_rhs_per_s": 3 * N * n / (t_op * 1e-3) / 1e9,
                   "kernel_gdof_rhs_per_s": 3 * N * n / (t_k * 1e-3) / 1e9,
                   "hbm_frac": B / (t_k * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "alu_frac": E * n * FLOPS_PER_ELEM_RHS / (t_k * 1e-3) / 1e12 / ALU_PEAK_TFLOPS}
            variants.append(rec)
            print(f"# {name} n={n}: matvec {t_op:.3f} ms, kernel {t_k:.3f} ms, "
                  f"{rec['gdof_rhs_per_s']:.1f} GDOF*RHS/s, HBM {rec['hbm_frac']:.2%}, ALU {rec['alu_frac']:.2%}",
                  file=sys.stderr, flush=True)
            if name == "f32" and n == 16:
                head = rec
            del xs, ys
            torch.cuda.empty_cache()

    # timed region of the headline step: FP32, 16 cases, y = K x
    n, dt = 16, torch.float32
    sets = 3
    xs = [torch.randn((N, 3, n), dtype=torch.float64, device="cuda").to(dt) for _ in range(sets)]
    ys = [torch.zeros((N, 3, n), dtype=dt, device="cuda") for _ in range(sets)]
    for i in range(args.warmup):
        gm.matvec(xs[i % sets], out=ys[i % sets])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        gm.matvec(xs[i % sets], out=ys[i % sets])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = 3 * N * n / (ms * 1e-3) / 1e9
    del xs, ys
    torch.cuda.empty_cache()

    t_k = head["ms_kernel"] * 1e-3
    B = kernel_bytes(N, Nv, E, 16, 4)
    hbm = {"bound": "hbm", "achieved": B / t_k / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": B / t_k / 1e9 / HBM_PEAK_GBS}
    alu = {"bound": "alu", "achieved": E * 16 * FLOPS_PER_ELEM_RHS / t_k / 1e12, "peak": ALU_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": E * 16 * FLOPS_PER_ELEM_RHS / t_k / 1e12 / ALU_PEAK_TFLOPS}
    roof, alt = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    traffic = load_traffic("ebe_p2_f32_n16")
    roof["traffic"] = None if traffic is None else traffic / 1e6  # MB per launch
    roof["kernel"] = "k_ebe_p2<float,16> (y += K x, 16 cases)"
    roof["kernel_ms"] = head["ms_kernel"]
    roof["algorithmic_bytes"] = B
    roof["algorithmic_flops"] = E * 16 * FLOPS_PER_ELEM_RHS

    line = {"metric": "EBE matvec GDOF*RHS/s (FP32, 16 cases) and % HBM peak; PCG solves/s mixed vs FP64",
            "value": value, "unit": "GDOF*RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"EBE matvec, unit cube {g}^3 hexes x 6 tets, jitter 0.2h, 3 layers",
                       "elements": E, "nodes": N, "dof": 3 * N, "nrhs": 16},
            "roofline": roof, "roofline_alt": alt, "variants": variants}
    if not args.no_solver:
        line["solver"] = solver_block(torch, ebe, meshgen)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(mesh, 16, args.cpu_elems)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
