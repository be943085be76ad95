"""The allocation-free product ebe_matvec_noalloc against ebe_matvec, called
through the C ABI: two calls in a row (the second on a smaller input) agree
with the allocating entry point within the product's rounding bound, and a
mesh whose staged sums exceed the fixed scratch array is refused."""
import numpy as np
import pytest
import torch

from helpers import kappa_max, oracle_K, parity_mesh, tol_factor
from paper_1710_08679_amd import ebe, meshgen

pytestmark = pytest.mark.gpu


def _pair(gm, m, K, dtype, nrhs, bc, seed):
    """(noalloc result, ebe_matvec result, bound) for one seeded input."""
    x = meshgen.random_vectors(meshgen.rng_for(91, seed), m.n_nodes, nrhs, dtype=dtype)
    xd = torch.from_numpy(x).cuda()
    y_na = torch.full_like(xd, float("nan"))
    gm.matvec_noalloc(xd, apply_bc=bc, out=y_na)
    y_ref = gm.matvec(xd, apply_bc=bc)
    torch.cuda.synchronize()
    xb = x.astype(np.float64)
    if bc:
        xb = xb * (1 - m.fixed[:, :, None])
    bound = (abs(K) @ np.abs(xb).reshape(-1, nrhs)).reshape(x.shape)
    return y_na.cpu().numpy().astype(np.float64), y_ref.cpu().numpy().astype(np.float64), bound


def _check(a, b, bound, dtype, kappa, what):
    # each side is within c kappa u |K||x| of K x, so they differ by at most twice that
    tol = 2.0 * tol_factor(dtype, kappa) * bound + 1e-300
    worst = float(np.max(np.abs(a - b) / tol))
    assert np.all(np.isfinite(a)), f"{what}: non-finite output"
    assert worst <= 1.0, f"{what}: max |noalloc - matvec| / bound = {worst:.3g}"


def test_noalloc_matches_matvec_two_calls(gpu_lib):
    big = parity_mesh(6, 5, 4, seed=3, bc=True)
    small = parity_mesh(3, 3, 2, seed=4, bc=True)
    gb, gs = ebe.Mesh.from_generated(big), ebe.Mesh.from_generated(small)
    kb, ks = kappa_max(big), kappa_max(small)
    Kb, Ks = oracle_K(big), oracle_K(small)
    print("noalloc: mesh 6x5x4 f32 n=8 bc, then mesh 3x3x2 f64 n=3 bc", flush=True)
    a, b, bound = _pair(gb, big, Kb, np.float32, 8, True, 0)
    _check(a, b, bound, np.float32, kb, "first call (6x5x4, FP32, 8 cases)")
    a, b, bound = _pair(gs, small, Ks, np.float64, 3, True, 1)
    _check(a, b, bound, np.float64, ks, "second call (3x3x2, FP64, 3 cases)")
    print("noalloc: mesh 6x5x4 f64 n=16 no bc, then f32 n=1 bc", flush=True)
    a, b, bound = _pair(gb, big, Kb, np.float64, 16, False, 2)
    _check(a, b, bound, np.float64, kb, "third call (6x5x4, FP64, 16 cases)")
    a, b, bound = _pair(gb, big, Kb, np.float32, 1, True, 3)
    _check(a, b, bound, np.float32, kb, "fourth call (6x5x4, FP32, 1 case)")


def test_noalloc_refuses_oversize_staging(gpu_lib):
    # 28^3 hexes: about 280k staged rows, 108 MB at FP64 with 16 cases (over
    # the 64 MiB scratch), 27 MB at FP32 with 8 cases (under it)
    m = meshgen.kuhn_mesh(28, 28, 28, jitter=0.2, rng=meshgen.rng_for(91, 50))
    gm = ebe.Mesh.from_generated(m)
    print("noalloc: 28^3 cube f64 n=16 (refused), f32 n=8 (accepted)", flush=True)
    x = torch.from_numpy(meshgen.random_vectors(meshgen.rng_for(91, 51), m.n_nodes, 16)).cuda()
    with pytest.raises(ebe.EbeError) as ei:
        gm.matvec_noalloc(x)
    assert ei.value.status == ebe.ERR_ARG and "scratch" in str(ei.value)
    x32 = torch.from_numpy(meshgen.random_vectors(meshgen.rng_for(91, 52), m.n_nodes, 8,
                                                  dtype=np.float32)).cuda()
    y_na = gm.matvec_noalloc(x32)
    y_ref = gm.matvec(x32)
    torch.cuda.synchronize()
    scale = float(torch.max(torch.abs(y_ref)))
    err = float(torch.max(torch.abs(y_na - y_ref))) / scale
    assert err < 1e-5, err
