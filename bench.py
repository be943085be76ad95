#!/usr/bin/env python3
"""Benchmark of the EBE hot path on one MI355X.

Workload (the EBE-matvec configuration): unit cube, 64^3 hexes x 6 = 1,572,864
straight 10-node tetrahedra, 2,146,689 nodes (6.44M DOF), interior corners
jittered by U(-0.2, 0.2) h, three horizontal layers (E = 1, 3, 8; nu = 0.25,
0.27, 0.30), seeded N(0, 1) input vectors.

A step is one y = K [x_1 .. x_16] product in FP32 (ebe_matvec), the product
the mixed-precision solver spends its time in.  `value` is DOF x RHS
processed per second (GDOF.RHS/s) with inputs resident in HBM, over the
`--steps` timed launches.  On the same JSON line: every (dtype, n) product
with the median and minimum of per-launch times, warm (rotating input sets)
and cold (after a 512 MB write that flushes the last-level cache); the
roofline of the headline product; whole solves per second of the multi-case
crust workload in each solver mode; the adjoint workload; the batched
uneven-mesh workload against the same solves one by one; and the CPU leg:
the oracle's assembled CSR product timed on a bounded sample, and the
oracle's own residual of every GPU solution.
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
# Published MI355X vector peaks: FP32 157.3 TFLOP/s (256 CU x 4 SIMD x 16
# lanes x 2.4 GHz x 2 flop per FMA x 2 for the packed two-wide FP32 FMA) and
# FP64 78.6 TFLOP/s.  The library is built with packed FP32 instructions off,
# so its plain FP32 FMAs can reach at most 78.6 TFLOP/s; both are reported.
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
PLAIN_FMA_PEAK_TFLOPS = 78.6
# Operation model of the element product: about 490 VALU operations per
# (element, case) (displacement-gradient coefficients 180, stresses 48,
# scaled stress sums 66, corner forces 60, edge forces 108, accumulation 30)
# plus about 80 per element (geometry), an FMA counting as one operation
# (two flops).
OPS_PER_ELEM_RHS = 490
OPS_PER_ELEM = 80


def product_flops(E, n):
    return 2.0 * E * (OPS_PER_ELEM_RHS * n + OPS_PER_ELEM)


def product_bytes(N, Nv, E, n, p):
    """Compulsory bytes of one EBE product: read x and write y once, the
    connectivity (10 int32), corner coordinates (3 doubles) and one material
    pair per element."""
    return 2 * 3 * N * n * p + 40 * E + 24 * Nv + 2 * E * p


def source_hash():
    h = hashlib.sha256()
    for f in ("ebe_kernels.hip", "pipe_kernel.h", "patch_common.h", "p2_element.h", "patches.cpp", "ebe_internal.h"):
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def time_each(fn, reps, warmup, torch, flush=None):
    """Per-launch milliseconds of fn over `reps` calls (an event pair around
    each call); flush() runs before each call, outside its events."""
    for i in range(warmup):
        fn(i)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i in range(reps):
        if flush is not None:
            flush()
        ev[i][0].record()
        fn(i)
        ev[i][1].record()
    torch.cuda.synchronize()
    return sorted(a.elapsed_time(b) for a, b in ev)


def stats_ms(ts):
    n = len(ts)
    med = ts[n // 2] if n % 2 else 0.5 * (ts[n // 2 - 1] + ts[n // 2])
    return {"median": med, "min": ts[0], "mean": sum(ts) / n, "reps": n}


# ---------------------------------------------------------------------------
# GPU blocks
# ---------------------------------------------------------------------------
def solver_block(torch, ebe, meshgen, modes):
    """Solves per second of the multi-case crust workload: 96x96x48 hexes x 6
    = 2,654,208 tetrahedra, 16 dislocation-pair cases, to 1e-8.  Returns the
    report and, for the CPU leg, the mesh, loads and host copies of the
    solutions."""
    m = meshgen.crust_mesh(96, 96, 48)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    gm = ebe.Mesh.from_generated(m)
    fd = torch.from_numpy(f).cuda()
    fixed = torch.from_numpy(m.fixed.astype(bool)).cuda()
    out = {"workload": "crust 96x96x48 hexes x 6 tets, 3 layers, 16 cases, tol 1e-8 (unsquared, max over cases)",
           "elements": m.n_elem, "dof": m.n_dof, "runs": []}
    sols = {}
    ref = None
    table = {"mixed_mg3": (ebe.PREC_MG3, ebe.MODE_MIXED), "mixed_mg3_fp16coarse": (ebe.PREC_MG3, ebe.MODE_MIXED),
             "mixed_mg3_deterministic": (ebe.PREC_MG3, ebe.MODE_MIXED),
             "fp64_mg3": (ebe.PREC_MG3, ebe.MODE_FP64),
             "mixed_mg2": (ebe.PREC_MG2, ebe.MODE_MIXED), "fp64_mg2": (ebe.PREC_MG2, ebe.MODE_FP64),
             "fp64_pcge": (ebe.PREC_PCGE, ebe.MODE_FP64)}
    for name in modes:
        precond, mode = table[name]
        half = int(name.endswith("fp16coarse"))
        det = int(name.endswith("deterministic"))
        torch.cuda.synchronize()
        tw = time.perf_counter()
        gm.solve(fd, precond=precond, mode=mode, tol=1e-8, coarse_half=half, deterministic=det)  # warm-up
        torch.cuda.synchronize()
        t_first = time.perf_counter() - tw
        times, u, st = [], None, None
        for _ in range(3):
            t0 = time.perf_counter()
            u, st = gm.solve(fd, precond=precond, mode=mode, tol=1e-8, coarse_half=half, deterministic=det)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = sorted(times)[1]
        r = fd.clone()
        r[fixed] = 0
        Ku = gm.matvec(u, apply_bc=True)
        res = float((torch.linalg.vector_norm((r - Ku).reshape(-1, 16), dim=0)
                     / torch.linalg.vector_norm(r.reshape(-1, 16), dim=0)).max())
        entry = {"mode": name, "seconds": dt, "seconds_min": min(times), "reps": len(times),
                 "first_solve_seconds": t_first, "solves_per_s": 16.0 / dt,
                 "outer_iters": st["outer_iters"], "inner_iters": st["inner_iters"],
                 "precond_used": st["precond_used"], "max_rel_res": st["max_rel_res"], "fp64_rel_res": res}
        if ref is None:
            ref = u.clone()
        else:
            entry["rel_diff_vs_first"] = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(u))
        out["runs"].append(entry)
        sols[name] = u.cpu().numpy()
        log(f"# solver {name}: median {dt:.3f} s of {len(times)}, {st}")
    fp64 = [r for r in out["runs"] if r["mode"].startswith("fp64")]
    mixed = [r for r in out["runs"] if r["mode"].startswith("mixed")]
    if fp64 and mixed:
        out["mixed_vs_fp64_speedup"] = {f"{a['mode']}/{b['mode']}": b["seconds"] / a["seconds"]
                                        for a in mixed for b in fp64}
    return out, (m, f, sols)


def greens_block(torch, ebe, meshgen, knots=(8, 4), step=4):
    """Green's functions of unit slips on a 45-degree fault in the crust
    (96x96x48 hexes x 6 tets; Section 5: sets of 16 cases) at surface
    stations, then the Eq. (5) inversion over 26 weights with the L-curve
    corner, on synthetic data from a known smooth slip with 1% noise."""
    import numpy as np
    m = meshgen.crust_mesh(96, 96, 48)
    flt = meshgen.dipping_fault(m, 0.5, (0.3, 1.7), (0.566, 1.556), knots)
    st = meshgen.surface_stations(m, step)
    gm = ebe.Mesh.from_generated(m)
    t0 = time.perf_counter()
    gf = ebe.Fault.from_generated(gm, flt)
    t_fault = time.perf_counter() - t0
    gf.greens_functions(st)  # warm-up: tuning, block Jacobi, level-2 set-up, workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G, stats = gf.greens_functions(st)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    rng = meshgen.rng_for(5, 40)
    # a smooth slip: a Gaussian patch over the basis grid, strike and dip parts
    ii, jj = np.meshgrid(np.arange(knots[0]), np.arange(knots[1]), indexing="ij")
    bump = np.exp(-((ii - 0.4 * knots[0]) ** 2 / (0.3 * knots[0]) ** 2 + (jj - 0.5 * knots[1]) ** 2 /
                    (0.4 * knots[1]) ** 2)).ravel()
    a_true = np.concatenate([bump, 0.5 * bump])
    Gh = G.cpu().numpy()
    clean = Gh @ a_true
    d = clean + 0.01 * np.abs(clean).max() * rng.standard_normal(clean.size)
    L = meshgen.laplacian_regularizer(*flt.knots)
    alphas = np.linalg.norm(Gh, 2) * np.logspace(-4, 1, 26)
    dd, Ld = torch.from_numpy(d).cuda(), torch.from_numpy(L).cuda()
    ebe.invert_lcurve(G, dd, Ld, alphas)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, rho, eta, curv, k = ebe.invert_lcurve(G, dd, Ld, alphas)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    ak = a[k].cpu().numpy()
    out = {"workload": f"crust 96x96x48 hexes x 6 tets, fault y - z = 0.5 (45 degrees), {flt.n_basis} unit-slip "
                       f"basis functions ({knots[0]} x {knots[1]} cubic B-splines x 2 directions) in sets of 16, "
                       f"{st.size} surface stations; inversion over 26 weights",
           "basis_functions": flt.n_basis, "stations": int(st.size), "fault_elements": int((flt.sides != 0).sum()),
           "fault_create_seconds": t_fault, "greens_seconds": t_g, "basis_functions_per_s": flt.n_basis / t_g,
           "sets": [{"outer_iters": x["outer_iters"], "max_rel_res": x["max_rel_res"], "status": x["status"]}
                    for x in stats],
           "inversion_ms": t_inv * 1e3, "corner_alpha_over_norm_G": float(alphas[k] / alphas[0] * 1e-4),
           "corner_slip_rel_err": float(np.linalg.norm(ak - a_true) / np.linalg.norm(a_true))}
    log(f"# greens: {flt.n_basis} basis functions in {t_g:.3f} s, inversion {t_inv * 1e3:.1f} ms, corner {k}, "
        f"slip error at the corner {out['corner_slip_rel_err']:.3g}")
    return out


FORM_NAMES = {0: "gather", 1: "staged", 2: "pipelined", 3: "assembled", 4: "coloured", 5: "deterministic"}


def curved_block(torch, ebe, meshgen, g, reps, warmup, straight):
    """Products on curved (isoparametric) elements: the matvec cube with every
    node moved by x -> (x + 0.25 x^2, y, z), so edge nodes leave their edge
    midpoints, through ebe_mesh_create_curved (the curved gather kernel).
    Per (dtype, n): median time against the straight mesh's, and an
    oracle-free check at full size (K applied to a linear field vanishes at
    interior nodes: a uniform stress is in equilibrium, exactly under this
    map)."""
    import numpy as np
    m = meshgen.quadratic_map(meshgen.matvec_mesh(g), 0.25)
    gm = ebe.Mesh.from_generated(m, curved=True)
    N = m.n_nodes
    out = {"workload": f"unit cube {g}^3 hexes x 6 tets mapped by x -> x + 0.25 x^2 (curved edges)",
           "elements": m.n_elem, "runs": []}
    for name, dt, n in (("f32", torch.float32, 16), ("f64", torch.float64, 16), ("f32", torch.float32, 4)):
        gm.autotune(0, dt, n)
        sets = 3
        xs = [torch.randn((N, 3, n), dtype=torch.float64, device="cuda").to(dt) for _ in range(sets)]
        ys = [torch.empty((N, 3, n), dtype=dt, device="cuda") for _ in range(sets)]
        warm = stats_ms(time_each(lambda i: gm.matvec(xs[i % sets], out=ys[i % sets]), reps, warmup, torch))
        ref = next((v["ms"] for v in straight if v["dtype"] == name and v["nrhs"] == n), None)
        rec = {"dtype": name, "nrhs": n, "ms": warm["median"], "warm_ms": warm,
               "gdof_rhs_per_s": 3 * N * n / (warm["median"] * 1e-3) / 1e9,
               "straight_ms": ref, "vs_straight": None if ref is None else warm["median"] / ref}
        out["runs"].append(rec)
        log(f"# curved {name} n={n}: {warm['median']:.3f} ms ({rec['gdof_rhs_per_s']:.1f} GDOF*RHS/s)"
            + ("" if ref is None else f", {rec['vs_straight']:.2f}x the straight mesh's {ref:.3f} ms"))
        del xs, ys
        torch.cuda.empty_cache()
    A = torch.from_numpy(meshgen.rng_for(2, 6).standard_normal((3, 3, 4))).cuda()
    xyz = torch.from_numpy(m.xyz).cuda()
    y = gm.matvec(torch.einsum("nd,cdr->ncr", xyz, A).contiguous()).abs().amax(dim=(1, 2)).cpu().numpy()
    # interior nodes whose elements all have one material (the layers' moduli
    # differ, and a uniform strain is in equilibrium only inside a layer)
    lo = np.full(N, np.inf)
    hi = np.full(N, -np.inf)
    ew = np.repeat(m.young, 10)
    np.minimum.at(lo, m.conn.ravel(), ew)
    np.maximum.at(hi, m.conn.ravel(), ew)
    inner = np.all((m.refined > 0) & (m.refined < 2 * g), axis=1) & (lo == hi)
    out["linear_field_check"] = {"interior_max_over_max": float(y[inner].max() / y.max()),
                                 "interior_nodes": int(inner.sum()),
                                 "what": "max |K u| at interior nodes inside one layer / max |K u|, u = A x linear "
                                         "(FP64, 4 cases)"}
    log(f"# curved linear-field check: {out['linear_field_check']}")
    return out


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
        log(f"# adjoint kernel {name} n={n}: {t:.3f} ms, {out['runs'][-1]['gelem_case_per_s']:.1f} Gelem*case/s")
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
    log(f"# adjoint misfit + gradient: {dt_s:.3f} s")
    return out


def batch_block(torch, ebe, meshgen, n_mesh, with_big, keep):
    """Batched uneven serving-size set: n_mesh crust meshes with log-uniform
    element counts in [5e4, 2e6] and 1..16 cases each, plus (with_big) the
    128x128x64 mesh with 16 cases; default solver options (mixed MG3) to
    1e-8, solved as one batch and then one after another.  Returns the
    report and, for the CPU leg, host copies of the `keep` smallest meshes'
    loads and batched solutions."""
    grids, nrhs = meshgen.batch_sizes(meshgen.rng_for(5, 0), n_mesh=n_mesh)
    if with_big:
        grids.append((128, 128, 64))
        nrhs.append(16)
    meshes, gms, fs = [], [], []
    for k, (gr, n) in enumerate(zip(grids, nrhs)):
        m = meshgen.crust_mesh(*gr)
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(5, 100 + k), nrhs=n)
        meshes.append(m)
        gms.append(ebe.Mesh.from_generated(m))
        fs.append(torch.from_numpy(f).cuda())
        log(f"# batch mesh {k}: grid {gr}, {m.n_elem} tets, {n} cases")
    opts = ebe.default_opts(tol=1e-8)
    # the default batch (concurrent solves on worker streams), then meshes of
    # up to 150k elements merged into block-diagonal systems
    ebe.batch_solve(gms, fs, opts=opts)  # warm-up: block Jacobi, level 2, workspaces, product forms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, st_b = ebe.batch_solve(gms, fs, opts=opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    info = {}
    ebe.batch_solve(gms, fs, opts=opts, merge_elems=150000, info=info)  # warm-up: the merged meshes are built
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st_m = ebe.batch_solve(gms, fs, opts=opts, merge_elems=150000)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    t0 = time.perf_counter()
    st_s = [gm.solve(f, opts=opts)[1] for gm, f in zip(gms, fs)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    cases = int(sum(nrhs))
    out = {"workload": f"{n_mesh} crust meshes, log-uniform 5e4..2e6 tets, 1..16 cases each"
                       + (" + 128x128x64 (16 cases)" if with_big else "") + ", mixed MG3 to 1e-8",
           "n_mesh": len(grids), "elements_total": int(sum(g.n_elem for g in gms)), "cases_total": cases,
           "batch_seconds": tb, "sequential_seconds": ts, "speedup": ts / tb,
           "merged_150k_seconds": tm, "merged_groups": info.get("groups"),
           "merged_meshes": int(sum(1 for g in info.get("group_of", []) if g >= 0)),
           "merged_max_rel_res": max(s["max_rel_res"] for s in st_m),
           "solves_per_s_batch": cases / tb, "solves_per_s_sequential": cases / ts,
           "max_rel_res": max(s["max_rel_res"] for s in st_b),
           "all_converged": all(s["status"] == ebe.OK for s in st_b + st_s)}
    log(f"# batch: {tb:.3f} s batched, {tm:.3f} s with small meshes merged ({info.get('groups')} groups), "
        f"{ts:.3f} s one by one, {cases} cases")
    small = sorted(range(len(meshes)), key=lambda i: meshes[i].n_elem)[:keep]
    kept = [(i, meshes[i], fs[i].cpu().numpy(), us[i].cpu().numpy()) for i in small]
    return out, kept


# ---------------------------------------------------------------------------
# CPU leg: the oracle
# ---------------------------------------------------------------------------
def cpu_spmm_baseline(mesh, n, n_elem_sample, reps=5):
    """The oracle's assembled operator on a bounded sample: K of the sub-mesh
    made of the first n_elem_sample elements (CSR, Eq. (3) assembled), then
    y = K X for X of shape (3 N_sub, n); the median of `reps` products.
    Assembly is timed separately."""
    import numpy as np
    from oracle import fem
    from paper_1710_08679_amd import meshgen
    conn = mesh.conn[:n_elem_sample]
    used = np.unique(conn)
    remap = -np.ones(mesh.n_nodes, np.int64)
    remap[used] = np.arange(used.size)
    sub = remap[conn]
    t0 = time.perf_counter()
    K = fem.assemble(mesh.xyz[used], sub, mesh.young[:n_elem_sample], mesh.poisson[:n_elem_sample],
                     n_nodes=used.size)
    t_asm = time.perf_counter() - t0
    X = meshgen.random_vectors(meshgen.rng_for(2, 99), used.size, n).reshape(3 * used.size, n)
    walls, cpus = [], []
    for _ in range(reps):
        t0, c0 = time.perf_counter(), time.process_time()
        K @ X
        walls.append(time.perf_counter() - t0)
        cpus.append(time.process_time() - c0)
    walls.sort()
    wall = walls[reps // 2]
    dof = 3 * used.size
    return {"value": dof * n / wall / 1e9, "unit": "GDOF*RHS/s", "cores": max(1, int(round(sum(cpus) / sum(walls)))),
            "kind": "oracle",
            "sample": f"oracle CSR product y = K X (scipy, FP64) of the sub-mesh of the first {n_elem_sample} of "
                      f"{mesh.n_elem} elements ({used.size} nodes, {K.nnz} nonzeros), n={n}: median of {reps} "
                      f"products {wall * 1e3:.1f} ms (min {walls[0] * 1e3:.1f} ms); assembly {t_asm:.1f} s",
            "assembly_seconds": t_asm, "host_cpus": os.cpu_count()}


def oracle_residuals(mesh, f, sols, threads):
    """max_j ||P (f_j - K u_j)|| / ||P f_j|| for each solution in `sols`,
    with the oracle's own element matrices (Eq. (3) by definition), in
    element chunks.  Each worker thread owns a node range and sums every
    element that touches it into that range only."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import fem
    names = list(sols)
    N = mesh.n_nodes
    n = f.shape[2]
    U = np.concatenate([sols[k].reshape(3 * N, n) for k in names], axis=1)  # (3N, modes * n)
    free = ~mesh.fixed.astype(bool).reshape(3 * N)
    fr = f.reshape(3 * N, n) * free[:, None]
    bounds = np.linspace(0, N, threads + 1).astype(np.int64)
    lo_el = mesh.conn.min(axis=1)
    hi_el = mesh.conn.max(axis=1)

    def work(w):
        n0, n1 = bounds[w], bounds[w + 1]
        cand = np.nonzero((hi_el >= n0) & (lo_el < n1))[0]
        touch = cand[((mesh.conn[cand] >= n0) & (mesh.conn[cand] < n1)).any(axis=1)]
        y = np.zeros((3 * (n1 - n0), U.shape[1]))
        for s in range(0, touch.size, 8000):
            es = touch[s:s + 8000]
            Ke = fem.element_stiffness_p2(mesh.xyz[mesh.conn[es]], mesh.young[es], mesh.poisson[es])
            dm = (3 * mesh.conn[es][:, :, None].astype(np.int64) + np.arange(3)).reshape(es.size, 30)
            ye = (Ke @ U[dm]).reshape(-1, U.shape[1])
            d = dm.ravel()
            keep = (d >= 3 * n0) & (d < 3 * n1)
            d, ye = d[keep] - 3 * n0, ye[keep]
            order = np.argsort(d, kind="stable")
            d, ye = d[order], ye[order]
            starts = np.concatenate([[0], np.nonzero(np.diff(d))[0] + 1])
            y[d[starts]] += np.add.reduceat(ye, starts, axis=0)
        r = fr[3 * n0:3 * n1, None, :] - (y * free[3 * n0:3 * n1, None]).reshape(-1, len(names), n)
        return (r * r).sum(axis=0), (fr[3 * n0:3 * n1] ** 2).sum(axis=0)

    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(work, range(threads)))
    rr = sum(p[0] for p in parts)
    ff = sum(p[1] for p in parts)
    rel = np.sqrt(rr / np.maximum(ff, 1e-300)[None, :])
    return {k: float(rel[i].max()) for i, k in enumerate(names)}


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=50, help="per-launch timings (median, min) of each product")
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--variants", default="f64:1,f64:4,f64:16,f32:1,f32:4,f32:16",
                    help="comma list of dtype:n products to time")
    ap.add_argument("--no-solver", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-greens", action="store_true")
    ap.add_argument("--no-curved", action="store_true")
    ap.add_argument("--solver-modes",
                    default="mixed_mg3,mixed_mg3_fp16coarse,mixed_mg3_deterministic,fp64_mg3,mixed_mg2,fp64_mg2,"
                            "fp64_pcge")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-elems", type=int, default=200000)
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle residual threads (0: min(16, cpus))")
    ap.add_argument("--batch", type=int, default=32, metavar="N_MESH",
                    help="uneven crust meshes in the batch workload (0: skip it)")
    ap.add_argument("--no-batch-big", action="store_true", help="leave the 128x128x64 mesh out of the batch")
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
    log(f"# workload {g}^3 x 6: E={E} N={N} DOF={3 * N}")

    flush_buf = torch.empty(128 << 20, dtype=torch.float32, device="cuda")  # 512 MB > the 256 MB MALL

    def flush():
        flush_buf.fill_(1.0)

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
        op = lambda i: gm.matvec(xs[i % sets], out=ys[i % sets])  # noqa: E731
        warm = stats_ms(time_each(op, args.reps, args.warmup, torch))
        cold = stats_ms(time_each(op, args.reps, 1, torch, flush=flush))
        t_op = warm["median"]
        B = product_bytes(N, Nv, E, n, p)
        F = product_flops(E, n)
        rec = {"dtype": name, "nrhs": n, "ms": t_op, "warm_ms": warm, "cold_ms": cold,
               "form": FORM_NAMES[gm.form(0, dt, n)],
               "autotune_ms": {FORM_NAMES[f]: t for f, t in enumerate(tms) if t >= 0},
               "gdof_rhs_per_s": 3 * N * n / (t_op * 1e-3) / 1e9,
               "hbm_frac": B / (t_op * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "valu_frac": F / (t_op * 1e-3) / 1e12 / VALU_PEAK_TFLOPS[name],
               "valu_frac_plain_fma": F / (t_op * 1e-3) / 1e12 / PLAIN_FMA_PEAK_TFLOPS}
        variants.append(rec)
        log(f"# {name} n={n} ({rec['form']}; tuning ms: "
            + " / ".join(f"{FORM_NAMES[f]} {t:.3f}" for f, t in enumerate(tms) if t >= 0) + "): "
            f"warm median {t_op:.3f} ms (min {warm['min']:.3f}), cold median {cold['median']:.3f} ms, "
            f"{rec['gdof_rhs_per_s']:.1f} GDOF*RHS/s, HBM {rec['hbm_frac']:.2%}, VALU {rec['valu_frac']:.2%} "
            f"(plain FMA {rec['valu_frac_plain_fma']:.2%})")
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
    if "f32:16" not in args.variants.split(","):
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
    F = product_flops(E, n)
    traffic = load_traffic(f"f32:16:{form}")
    roof = {"bound": "alu", "achieved": F / t / 1e12, "peak": VALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
            "frac": F / t / 1e12 / VALU_PEAK_TFLOPS["f32"], "traffic": traffic,
            "frac_of_plain_fma_peak": F / t / 1e12 / PLAIN_FMA_PEAK_TFLOPS,
            "ops_model": f"E*({OPS_PER_ELEM_RHS}n+{OPS_PER_ELEM}) VALU ops per product, FMA = 2 flops",
            "kernel": f"EBE product FP32 n=16, {form} form (ebe_matvec: "
                      + ("one k_ebe_pipe launch per patch colour" if form == "coloured" else
                         "patch kernel + shared-node pass") + ")",
            "launches_per_product": gm.patch_info(0)["colours"] if form == "coloured" else 2,
            "ms_per_product": ms_events,
            "algorithmic_flops": F, "algorithmic_bytes": B,
            "hbm": {"achieved": B / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": B / t / 1e9 / HBM_PEAK_GBS}}
    if traffic is not None:
        roof["traffic_over_algorithmic"] = traffic / B
    head = next((v for v in variants if v["dtype"] == "f32" and v["nrhs"] == 16), None)
    if head is not None:
        roof["warm_ms"], roof["cold_ms"] = head["warm_ms"], head["cold_ms"]

    line = {"metric": "EBE matvec GDOF*RHS/s (FP32, 16 cases) and % HBM peak; PCG solves/s mixed vs FP64",
            "value": value, "unit": "GDOF*RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"EBE matvec, unit cube {g}^3 hexes x 6 tets, jitter 0.2h, 3 layers, 16 cases",
                       "elements": E, "nodes": N, "dof": 3 * N, "nrhs": 16},
            "roofline": roof, "variants": variants}
    del flush_buf
    torch.cuda.empty_cache()
    if not args.no_curved:
        line["curved"] = curved_block(torch, ebe, meshgen, g, args.reps, args.warmup, variants)
        torch.cuda.empty_cache()
    solved = None
    if not args.no_solver:
        line["solver"], solved = solver_block(torch, ebe, meshgen, args.solver_modes.split(","))
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        line["adjoint"] = adjoint_block(torch, ebe, meshgen, args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_greens:
        line["greens"] = greens_block(torch, ebe, meshgen)
        torch.cuda.empty_cache()
    kept = []
    if args.batch > 0:
        line["batch"], kept = batch_block(torch, ebe, meshgen, args.batch, not args.no_batch_big, keep=4)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_spmm_baseline(mesh, 16, args.cpu_elems)
        log(f"# cpu baseline: {line['cpu_baseline']['sample']}")
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        if solved is not None:
            m3, f3, sols = solved
            t0 = time.perf_counter()
            rel = oracle_residuals(m3, f3, sols, threads)
            for r in line["solver"]["runs"]:
                r["oracle_rel_res"] = rel[r["mode"]]
            line["solver"]["oracle_check"] = (f"max_j ||P(f_j - K u_j)|| / ||P f_j|| with the oracle's element "
                                              f"matrices on all {m3.n_elem} elements, {threads} threads, "
                                              f"{time.perf_counter() - t0:.1f} s")
            log(f"# oracle residuals of the crust solutions: {rel}")
        if kept:
            checks = []
            for i, mk, fk, uk in kept:
                rel = oracle_residuals(mk, fk, {"batch": uk}, threads)["batch"]
                checks.append({"mesh": i, "elements": mk.n_elem, "nrhs": int(fk.shape[2]), "oracle_rel_res": rel})
            line["batch"]["oracle_check"] = checks
            log(f"# oracle residuals of batch solutions: {checks}")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
