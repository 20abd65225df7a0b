"""GPU tests of the batched solve and of HIP-graph capture.

A batch runs, per pass, one launch per group of equal-length members with the
same kernel variant, using the kernels ps_solve uses: every member must equal
ps_solve's result for its plan bitwise, and match the oracle at the parity
tolerance.  A captured graph must replay the eager result bitwise, with the
program's own eager work and synchronisations between replays.
"""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from paper_2409_02294_amd import inputs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_2409_02294_amd import solver as S

def _make(prec, sizes, seed, variants=None):
    dt = torch.float64 if prec == "f64" else torch.float32
    solvers, rhos = [], []
    for i, n in enumerate(sizes):
        s = S.Solver(n, 1.0 / n, prec)
        if variants is not None and variants[i] is not None:
            for k, v in enumerate(variants[i]):
                S.ps_plan_set_variant(s.plan, k, v)
        rng = np.random.default_rng(seed + i)
        blobs = inputs.draw_blobs(rng, int(rng.integers(4, 33)), centre=(0.1, 0.9), sigma=(0.03, 0.08))
        rho = torch.from_numpy(inputs.blob_density(n, blobs)).to("cuda", dt)
        solvers.append(s)
        rhos.append(rho)
    return solvers, rhos


@pytest.mark.parametrize("prec", ["f32", "f64", "f32_split"])
def test_batch_matches_single_solves(prec):
    sizes = [32, 128, 48, 64, 16, 96, 128, 32, 64, 24, 8, 48]
    solvers, rhos = _make(prec, sizes, 4000)
    eager = [s(r) for s, r in zip(solvers, rhos)]
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    for n, a, b in zip(sizes, outs, eager):
        assert torch.equal(a, b), n
    # every member against the oracle
    tol = 1e-12 if prec == "f64" else 1e-6
    for n, a, r in zip(sizes, outs, rhos):
        ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
        err = oracle.rel_l2(a.double().cpu().numpy(), ref)
        assert err <= tol, (n, err)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_of_five_smooth_lengths(prec):
    # radices 5, 3 x 3, 10, 15, 6, 12, 20 inside one batch, two members per length
    sizes = [40, 72, 80, 120, 144, 40, 96, 160, 120, 72]
    solvers, rhos = _make(prec, sizes, 4200)
    eager = [s(r) for s, r in zip(solvers, rhos)]
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    for n, a, b in zip(sizes, outs, eager):
        assert torch.equal(a, b), n
    tol = 1e-12 if prec == "f64" else 1e-6
    for n, a, r in zip(sizes[:5], outs[:5], rhos[:5]):
        ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
        assert oracle.rel_l2(a.double().cpu().numpy(), ref) <= tol, n


def test_batch_with_large_member():
    # two n = 256 members share one launch of the persistent z pass (FP32 default there)
    sizes = [256, 32, 64, 128, 256]
    solvers, rhos = _make("f32", sizes, 4100)
    eager = [s(r) for s, r in zip(solvers, rhos)]
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    for n, a, b in zip(sizes, outs, eager):
        assert torch.equal(a, b), n


@pytest.mark.parametrize("prec", ["f32", "f32_split"])
def test_batch_mixed_variants(prec):
    # equal lengths with different kernel variants split into separate launches
    sizes = [128, 128, 128, 64, 64, 256, 256]
    if prec == "f32":
        var = [None, [0, 0, 0, 0, 0], [0, 0, 1, 0, 0], None, [0, 0, 0, 0, 0], [1, 1, 2, 1, 1], [0, 0, 1, 0, 0]]
    else:
        var = [None, [0, 0, 0, 0, 0], [0, 0, 1, 0, 0], None, [0, 0, 0, 0, 0], None, [0, 0, 0, 0, 0]]
    solvers, rhos = _make(prec, sizes, 4150, var)
    if prec == "f32_split":  # product terms differ per plan too
        S.ps_plan_set_variant(solvers[1].plan, 5, 3)
        S.ps_plan_set_variant(solvers[5].plan, 5, 3)
    # and z tiles: members 3 and 4 share every pass variant but the z tile
    v3 = solvers[3].info()
    for k in range(5):
        S.ps_plan_set_variant(solvers[4].plan, k, v3["variant"][k])
    S.ps_plan_set_variant(solvers[4].plan, 6, 1 - v3["z_tile"])
    eager = [s(r) for s, r in zip(solvers, rhos)]
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    for n, a, b in zip(sizes, outs, eager):
        assert torch.equal(a, b), n
    # a changed variant is a new batch: new records, same results as ps_solve
    S.ps_plan_set_variant(solvers[0].plan, 2, 0)
    eager0 = solvers[0](rhos[0])
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], eager0)


def test_batch_repeat_and_reorder():
    sizes = [64, 32, 96]
    solvers, rhos = _make("f32", sizes, 4200)
    first = [o.clone() for o in S.solve_batched(solvers, rhos)]
    again = S.solve_batched(solvers, rhos)  # same list: no upload
    for a, b in zip(first, again):
        assert torch.equal(a, b)
    # a different order is a different batch (new member records)
    rev = S.solve_batched(solvers[::-1], rhos[::-1])
    for a, b in zip(first, rev[::-1]):
        assert torch.equal(a, b)


def test_batch_argument_errors():
    solvers, rhos = _make("f32", [16, 16], 4300)
    lib = S.load()
    with pytest.raises(S.PSError) as e:
        S.ps_solve_batched([solvers[0].plan, solvers[0].plan], [rhos[0].data_ptr()] * 2,
                           [torch.empty_like(rhos[0]).data_ptr(), torch.empty_like(rhos[0]).data_ptr()], 0)
    assert e.value.status == S.PS_ERR_INVALID
    out = torch.empty_like(rhos[0])
    with pytest.raises(S.PSError) as e:  # both outputs in the same array
        S.ps_solve_batched([s.plan for s in solvers], [r.data_ptr() for r in rhos], [out.data_ptr()] * 2, 0)
    assert e.value.status == S.PS_ERR_INVALID
    f64 = S.Solver(16, 1.0 / 16, "f64")
    with pytest.raises(S.PSError) as e:  # mixed arithmetic
        S.ps_solve_batched([solvers[0].plan, f64.plan], [rhos[0].data_ptr(), rhos[1].data_ptr()],
                           [torch.empty_like(rhos[0]).data_ptr(), torch.empty(16 ** 3, dtype=torch.float64, device="cuda").data_ptr()], 0)
    assert e.value.status == S.PS_ERR_INVALID


def _replay_check(g, outs, eager, work):
    for rep in range(3):
        work()  # eager work of the program between replays
        torch.cuda.synchronize()
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), f"replay {rep} differs"


def test_graph_replay_single_solve():
    n = 64
    s = S.Solver(n, 1.0 / n, "f32")
    rho = torch.from_numpy(inputs.make_density(n, 8, 11, sigma=(0.03, 0.08))).to("cuda", torch.float32)
    out = torch.empty_like(rho)
    s(rho, out)
    torch.cuda.synchronize()
    eager = out.clone()
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        s(rho, out)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            s.solve(rho, out)
    _replay_check(g, [out], [eager], lambda: s(rho * 2.0))


def test_graph_replay_batched():
    sizes = [32, 48, 64, 96, 128, 32, 64]
    solvers, rhos = _make("f32", sizes, 4400)
    outs = [torch.empty_like(r) for r in rhos]
    S.solve_batched(solvers, rhos, outs)  # first call uploads the member records
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        S.solve_batched(solvers, rhos, outs)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            S.solve_batched(solvers, rhos, outs)
    _replay_check(g, outs, eager, lambda: [s(r) for s, r in zip(solvers, rhos)])


def test_capture_of_new_batch_is_refused():
    sizes = [32, 16]
    solvers, rhos = _make("f32", sizes, 4500)
    outs = [torch.empty_like(r) for r in rhos]
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    status = None
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            outs[0].add_(1.0)
            try:
                S.solve_batched(solvers, rhos, outs)
            except S.PSError as e:
                status = e.status
    assert status == S.PS_ERR_CAPTURE


# ---------------------------------------------------------------------------
# The two batched workloads themselves, member by member against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32_split", "f32"])
def test_batched_workload_matches_oracle(prec):
    # 96 solves, N in {32, 48, 64, 96, 128} (seeded), 4-32 blobs each, one batched call
    dens = inputs.batched_workload(96, 4000)
    solvers = [S.Solver(d.shape[0], 1.0 / d.shape[0], prec) for d in dens]
    rhos = [torch.from_numpy(d).to("cuda", torch.float32) for d in dens]
    outs = S.solve_batched(solvers, rhos)
    torch.cuda.synchronize()
    worst_l2 = worst_max = 0.0
    for s, r, o in zip(solvers, rhos, outs):
        rho64 = r.double().cpu().numpy()
        ref = oracle.fft_conv(rho64, 1.0 / s.n)
        got = o.double().cpu().numpy()
        l2, mx = oracle.rel_l2(got, ref), oracle.rel_max(got, ref)
        assert l2 <= 1e-6, (s.n, l2)
        worst_l2, worst_max = max(worst_l2, l2), max(worst_max, mx)
    print(f"batched workload {prec}: worst member relL2 {worst_l2:.2e}, relMax {worst_max:.2e}", flush=True)


@pytest.mark.parametrize("prec", ["f32_split", "f32"])
def test_nested_workload_steps(prec):
    # 384^3 coarse level + two 128^3 levels refined by 2, drifting blobs: steps 0 and 199
    geometry, sets = inputs.nested_workload(200)
    solvers = [S.Solver(n, dx, prec) for (n, dx, _) in geometry]
    for t in (0, 199):
        dens = [inputs.blob_density(n, sets[t], dx, origin) for (n, dx, origin) in geometry]
        rhos = [torch.from_numpy(d).to("cuda", torch.float32) for d in dens]
        outs = S.solve_batched(solvers, rhos)
        torch.cuda.synchronize()
        for lv, ((n, dx, _), r, o) in enumerate(zip(geometry, rhos, outs)):
            rho64 = r.double().cpu().numpy()
            if n <= 128:
                ref = oracle.fft_conv(rho64, dx)
                l2 = oracle.rel_l2(o.double().cpu().numpy(), ref)
                print(f"nested {prec} step {t} level {lv} ({n}^3): relL2 {l2:.2e}", flush=True)
                assert l2 <= 1e-6
            else:
                rng = np.random.default_rng(t)
                cells = rng.integers(0, n, (24, 3))
                cells[:2] = [[n // 2, n // 2, n // 2], [0, n - 1, n // 3]]
                ref = oracle.direct_sum_cells(rho64, cells, dx)
                idx = torch.from_numpy(cells).to("cuda", torch.long)
                got = o[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
                err = float(np.abs(got - ref).max() / np.abs(ref).max())
                print(f"nested {prec} step {t} level {lv} ({n}^3): sampled relMax {err:.2e}", flush=True)
                assert err <= 1e-6
